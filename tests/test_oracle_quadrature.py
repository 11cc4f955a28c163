"""Pins of the oracle's quadrature and panel integrals against mathematics.

* Triangle rules: exact monomial integrals a! b! / (a+b+2)! on the reference
  triangle up to the rule's degree.
* Semi-analytic self integral: the closed form of the Laplace integral and
  an independent Duffy-transformed 1-D integral (scipy ``quad``) for Laplace
  and Yukawa.
* Near-singular entries: adaptive 2-D integration (scipy ``dblquad``) of the
  same panel integral.
* Row sums on a sphere of radius a: sum_j K_L = -1/2, sum_j V_L = a,
  sum_j V_Y = (1 - exp(-2 kappa a)) / (2 kappa),
  sum_j K_Y = -(1 - (1 + kappa a) exp(-2 kappa a)) / (2 kappa a).
"""

import math

import numpy as np
import pytest
from scipy import integrate

import synth
from oracle.geometry import gauss_points, panels
from oracle.integrals import panel_integrals, self_integral, self_integral_laplace_exact
from oracle.quadrature import gauss_legendre, rule_degree, triangle_rule


@pytest.mark.parametrize("k", [1, 3, 4, 7, 19])
def test_triangle_rule_exact_on_monomials(k):
    bary, w = triangle_rule(k)
    assert abs(w.sum() - 1.0) < 1e-14
    assert np.all(bary >= 0.0) and np.allclose(bary.sum(axis=1), 1.0, atol=1e-15)
    deg = rule_degree(k)
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
            quad = 0.5 * np.sum(w * bary[:, 1] ** a * bary[:, 2] ** b)
            assert abs(quad - exact) <= 1e-14 * max(1.0, 1.0 / exact) * exact + 1e-16
    # one degree higher is not integrated exactly (the degree is not overstated)
    errs = []
    for a in range(deg + 2):
        b = deg + 1 - a
        exact = math.factorial(a) * math.factorial(b) / math.factorial(a + b + 2)
        errs.append(abs(0.5 * np.sum(w * bary[:, 1] ** a * bary[:, 2] ** b) - exact))
    assert max(errs) > 1e-9


def test_gauss_legendre():
    for n in (1, 3, 5, 8):
        x, w = gauss_legendre(n)
        for p in range(2 * n):
            exact = 0.0 if p % 2 else 2.0 / (p + 1)
            assert abs(np.sum(w * x ** p) - exact) < 1e-13


def _one_panel():
    v = np.array([[0.0, 0.0, 0.0], [1.3, 0.1, 0.0], [0.2, 0.9, 0.0]])
    return panels(v, np.array([[0, 1, 2]]))


def _duffy_self(p, j, kappa):
    """int over panel j of G(x_j, y) dA_y by a Duffy split at x_j: for the
    sub-triangle (x, A, B), y = x + u (A - x + v (B - A)), dA = u J du dv,
    and the u-integral is done in closed form; v by adaptive quad."""
    x = p.centre[j]
    vs = [p.v0[j], p.v1[j], p.v2[j]]
    total = 0.0
    for a, b in ((0, 1), (1, 2), (2, 0)):
        A, B = vs[a], vs[b]
        J = np.linalg.norm(np.cross(A - x, B - A))

        def f(v):
            rho = np.linalg.norm(A - x + v * (B - A))
            if kappa == 0.0:
                return 1.0 / rho
            return -math.expm1(-kappa * rho) / (kappa * rho * rho)

        total += J / (4.0 * math.pi) * integrate.quad(f, 0.0, 1.0, epsabs=1e-15, epsrel=1e-13, limit=200)[0]
    return total


def test_self_integral_laplace_closed_form():
    p = _one_panel()
    exact = self_integral_laplace_exact(p, [0])[0]
    duffy = _duffy_self(p, 0, 0.0)
    assert abs(exact - duffy) < 1e-13 * abs(exact)
    # the N_k-point angular rule converges to it
    assert abs(self_integral(p, [0], 0.0, 40)[0] - exact) < 1e-13 * abs(exact)
    e5 = abs(self_integral(p, [0], 0.0, 5)[0] - exact)
    e3 = abs(self_integral(p, [0], 0.0, 3)[0] - exact)
    assert e5 < 1e-3 * abs(exact) and e5 < e3


@pytest.mark.parametrize("kappa", [0.125, 1.0, 3.0])
def test_self_integral_yukawa_duffy(kappa):
    p = _one_panel()
    duffy = _duffy_self(p, 0, kappa)
    assert abs(self_integral(p, [0], kappa, 40)[0] - duffy) < 1e-12 * abs(duffy)
    assert abs(self_integral(p, [0], kappa, 5)[0] - duffy) < 1e-3 * abs(duffy)
    # small kappa approaches the Laplace value
    lap = self_integral_laplace_exact(p, [0])[0]
    assert abs(self_integral(p, [0], 1e-7, 40)[0] - lap) < 1e-6 * lap


def _brute(x, p, j, kappa, kind):
    v0, v1, v2 = p.v0[j], p.v1[j], p.v2[j]
    e1, e2 = v1 - v0, v2 - v0
    jac = np.linalg.norm(np.cross(e1, e2))
    n = p.normal[j]

    def f(t, s):
        y = v0 + s * e1 + t * e2
        d = x - y
        R = math.sqrt(d @ d)
        if kind == "V":
            g = math.exp(-kappa * R) / (4 * math.pi * R)
        else:
            g = (n @ d) * (1 + kappa * R) * math.exp(-kappa * R) / (4 * math.pi * R ** 3)
        return g * jac

    return integrate.dblquad(f, 0.0, 1.0, 0.0, lambda s: 1.0 - s, epsabs=1e-15, epsrel=1e-12)[0]


@pytest.mark.parametrize("kappa", [0.0, 0.5])
def test_near_singular_entries_vs_adaptive(kappa):
    """Near-zone entries approach the adaptive 2-D integral as the rule grows
    (4 -> 7 -> 19 points) and the 19-point rule is within its expected error
    once the target is more than 0.8 L from the panel centre."""
    v, f = synth.geodesic_sphere("oct", 2, 1.0)
    p = panels(v, f)
    X = p.centre
    res = {kf: panel_integrals(X, p, kappa, k=4, k_fine=kf, thres=2.0, nk=5,
                               self_idx=np.arange(p.n)) for kf in (4, 7, 19)}
    dist = np.linalg.norm(X[:, None] - p.centre[None], axis=2)
    near = (dist < 2.0 * p.length[None, :]) & (dist > 0)
    ii, jj = np.nonzero(near)
    assert len(ii) > 10
    for i, j in list(zip(ii, jj))[:12]:
        bv = _brute(X[i], p, j, kappa, "V")
        bk = _brute(X[i], p, j, kappa, "K")
        err = {kf: max(abs(res[kf][0][i, j] - bv), abs(res[kf][1][i, j] - bk)) / abs(bv)
               for kf in res}
        assert err[19] < min(err[7], err[4])
        if dist[i, j] > 0.8 * p.length[j]:
            assert err[19] < 5e-5
        assert err[19] < 2e-2


def test_far_entries_match_k_point_rule():
    """Entries outside the near zone use the K-point rule unchanged."""
    v, f = synth.geodesic_sphere("oct", 3, 2.0)
    p = panels(v, f)
    X = np.array([[0.05, 0.02, 0.03]])
    V, K = panel_integrals(X, p, 0.3, k=4, thres=1.0)
    y, W = gauss_points(p, 4)
    d = X[0] - y
    R = np.linalg.norm(d, axis=2)
    Vr = np.sum(W * np.exp(-0.3 * R) / (4 * math.pi * R), axis=1)
    assert np.allclose(V[0], Vr, rtol=1e-14, atol=0)
    Kr = np.sum(W * np.einsum("jkc,jc->jk", d, p.normal) * (1 + 0.3 * R)
                * np.exp(-0.3 * R) / (4 * math.pi * R ** 3), axis=1)
    assert np.allclose(K[0], Kr, rtol=1e-12, atol=1e-16)


@pytest.mark.parametrize("kappa", [0.0, 0.125])
def test_row_sums_on_sphere(kappa):
    a = 4.0
    errs = []
    for nu in (4, 8):
        v, f = synth.geodesic_sphere("oct", nu, a)
        p = panels(v, f)
        rows = np.arange(0, p.n, max(1, p.n // 24))
        V, K = panel_integrals(p.centre[rows], p, kappa, self_idx=rows)
        sv, sk = V.sum(axis=1), K.sum(axis=1)
        if kappa == 0.0:
            ev, ek = a, -0.5
        else:
            ev = -math.expm1(-2 * kappa * a) / (2 * kappa)
            ek = -(1 - (1 + kappa * a) * math.exp(-2 * kappa * a)) / (2 * kappa * a)
        errs.append((np.max(np.abs(sv - ev)) / ev, np.max(np.abs(sk - ek)) / abs(ek)))
    (ev8, ek8) = errs[1]
    assert ev8 < 1e-2 and ek8 < 1e-2
    # both row sums converge under refinement
    assert errs[1][0] < errs[0][0] and errs[1][1] < errs[0][1]
