"""Green's functions and panel integrals (oracle, test infrastructure only).

Green's functions carry the 1/(4 pi) of Eq. nBEM:
    Laplace  G_L(x, y) = 1 / (4 pi R)
    Yukawa   G_Y(x, y) = exp(-kappa R) / (4 pi R),   R = |x - y|,
and the double layer takes the normal derivative at the source point y:
    n . grad_y G = n . (x - y) (1 + kappa R) exp(-kappa R) / (4 pi R^3).

For a target x and a panel j the oracle forms
    V = int_{panel j} G(x, y) dA_y,     K = int_{panel j} n_j . grad_y G(x, y) dA_y
(Eq. matel) with the rule picked as in sec. 2.3 (treecode-accelerated BEM)
and the lysozyme parameter table of sec. 3:
  * x is the collocation point of panel j itself: the semi-analytic rule of
    Zhu et al. -- the panel is split at x into three sub-triangles, the
    radial integral is done in closed form and the angle by N_k-point
    Gauss-Legendre per sub-triangle; K = 0 because x lies in the flat panel;
  * |x - centre_j| < thres * L_j: the K_fine-point rule;
  * otherwise: the K-point rule.
"""

from __future__ import annotations

import math

import numpy as np

from .geometry import Panels, gauss_points
from .quadrature import gauss_legendre

FOUR_PI = 4.0 * math.pi


def green(R, kappa):
    if kappa == 0.0:
        return 1.0 / (FOUR_PI * R)
    return np.exp(-kappa * R) / (FOUR_PI * R)


def green_dn(dn, R, kappa):
    """n . grad_y G with dn = n . (x - y)."""
    if kappa == 0.0:
        return dn / (FOUR_PI * R ** 3)
    return dn * (1.0 + kappa * R) * np.exp(-kappa * R) / (FOUR_PI * R ** 3)


def green_dkappa(R, kappa):
    """d G_Y / d kappa = -exp(-kappa R) / (4 pi)."""
    return -np.exp(-kappa * R) / FOUR_PI


def green_dn_dkappa(dn, R, kappa):
    """d (n . grad_y G_Y) / d kappa = -kappa n.(x - y) exp(-kappa R) / (4 pi R)."""
    return -kappa * dn * np.exp(-kappa * R) / (FOUR_PI * R)


def _radial(rho, kappa, kind):
    """Closed-form radial integral int_0^rho G(r) r dr of the polar rule."""
    if kind == "value":
        if kappa == 0.0:
            return rho / FOUR_PI
        return -np.expm1(-kappa * rho) / (FOUR_PI * kappa)
    # d/d kappa of the line above
    if kappa == 0.0:
        return -rho * rho / (2.0 * FOUR_PI)
    e = np.exp(-kappa * rho)
    return (kappa * rho * e + np.expm1(-kappa * rho)) / (FOUR_PI * kappa * kappa)


def _edge_frames(p: Panels, idx, x):
    """For every panel in ``idx`` and each of its 3 edges: the distance h from
    x to the edge line and the angles (from the foot of the perpendicular)
    of the edge end points."""
    vs = (p.v0[idx], p.v1[idx], p.v2[idx])
    out = []
    for a, b in ((0, 1), (1, 2), (2, 0)):
        A, B = vs[a], vs[b]
        e = B - A
        lab = np.linalg.norm(e, axis=1)
        e = e / lab[:, None]
        t = np.einsum("ij,ij->i", x - A, e)
        foot = A + t[:, None] * e
        h = np.linalg.norm(x - foot, axis=1)
        ta = np.arctan2(-t, h)
        tb = np.arctan2(lab - t, h)
        out.append((h, ta, tb))
    return out


def self_integral(p: Panels, idx, kappa, nk, kind="value"):
    """Semi-analytic V of each panel in ``idx`` at its own centre.

    int_panel G dA = sum over sub-triangles int_{ta}^{tb} R(rho_max(t)) dt,
    rho_max(t) = h / cos t, R(rho) = int_0^rho G(r) r dr in closed form.
    """
    idx = np.asarray(idx)
    x = p.centre[idx]
    gx, gw = gauss_legendre(nk)
    total = np.zeros(len(idx))
    for h, ta, tb in _edge_frames(p, idx, x):
        half = 0.5 * (tb - ta)
        mid = 0.5 * (tb + ta)
        th = mid[:, None] + half[:, None] * gx[None, :]
        rho = h[:, None] / np.cos(th)
        total += half * np.sum(gw[None, :] * _radial(rho, kappa, kind), axis=1)
    return total


def self_integral_laplace_exact(p: Panels, idx):
    """Closed form of the Laplace self integral: sum h/(4 pi) [ln(sec t + tan t)]."""
    idx = np.asarray(idx)
    x = p.centre[idx]
    total = np.zeros(len(idx))
    for h, ta, tb in _edge_frames(p, idx, x):
        f = lambda t: np.log(1.0 / np.cos(t) + np.tan(t))
        total += h / FOUR_PI * (f(tb) - f(ta))
    return total


def _rule_sums(X, y, W, normal, kappa, kind):
    with np.errstate(divide="ignore", invalid="ignore"):
        return _rule_sums_raw(X, y, W, normal, kappa, kind)


def _rule_sums_raw(X, y, W, normal, kappa, kind):
    """K-point sums over panels for targets X: returns V, K (m, n)."""
    d = X[:, None, None, :] - y[None, :, :, :]  # (m, n, K, 3)
    R = np.sqrt(np.einsum("mnkc,mnkc->mnk", d, d))
    dn = np.einsum("mnkc,nc->mnk", d, normal)
    if kind == "value":
        g = green(R, kappa)
        gd = green_dn(dn, R, kappa)
    else:
        g = green_dkappa(R, kappa)
        gd = green_dn_dkappa(dn, R, kappa)
    return np.einsum("mnk,nk->mn", g, W), np.einsum("mnk,nk->mn", gd, W)


def panel_integrals(X, p: Panels, kappa, k=4, k_fine=19, thres=2.0, nk=5,
                    self_idx=None, kind="value", chunk_pairs=3_000_000):
    """Dense V, K (m, n) for targets X against all panels of ``p``.

    ``self_idx[i]`` is the panel whose centre is X[i] (or -1).  ``kind`` is
    "value" or "dkappa" (derivative of the Yukawa kernels with respect to
    kappa, used by the gradient oracle).
    """
    X = np.asarray(X, dtype=np.float64).reshape(-1, 3)
    m, n = len(X), p.n
    if self_idx is None:
        self_idx = -np.ones(m, dtype=np.int64)
    self_idx = np.asarray(self_idx)
    y, W = gauss_points(p, k)
    yf, Wf = gauss_points(p, k_fine)
    V = np.empty((m, n))
    K = np.empty((m, n))
    step = max(1, chunk_pairs // max(1, n * k))
    for s in range(0, m, step):
        e = min(m, s + step)
        Xc = X[s:e]
        Vc, Kc = _rule_sums(Xc, y, W, p.normal, kappa, kind)
        dist = np.linalg.norm(Xc[:, None, :] - p.centre[None, :, :], axis=2)
        near = dist < thres * p.length[None, :]
        rows = np.arange(s, e)
        own = self_idx[s:e]
        has_self = own >= 0
        near[np.nonzero(has_self)[0], own[has_self]] = False
        ii, jj = np.nonzero(near)
        for c0 in range(0, len(ii), max(1, chunk_pairs // k_fine)):
            c1 = min(len(ii), c0 + max(1, chunk_pairs // k_fine))
            a, b = ii[c0:c1], jj[c0:c1]
            d = Xc[a][:, None, :] - yf[b]  # (q, Kf, 3)
            R = np.linalg.norm(d, axis=2)
            dn = np.einsum("qkc,qc->qk", d, p.normal[b])
            if kind == "value":
                g, gd = green(R, kappa), green_dn(dn, R, kappa)
            else:
                g, gd = green_dkappa(R, kappa), green_dn_dkappa(dn, R, kappa)
            Vc[a, b] = np.sum(g * Wf[b], axis=1)
            Kc[a, b] = np.sum(gd * Wf[b], axis=1)
        if np.any(has_self):
            li = np.nonzero(has_self)[0]
            Vc[li, own[li]] = self_integral(p, own[li], kappa, nk, kind)
            Kc[li, own[li]] = 0.0
        V[s:e] = Vc
        K[s:e] = Kc
        del rows
    return V, K
