"""Closed-form solvation energies for spheres (oracle pins; test only).

These are exact solutions of the PDE system of sec. 2.1 (Eq. pde) for
spherical geometry; they pin the oracle's units, 4 pi factors, epsilon ratio
and sign conventions.  Energies in kJ/mol, lengths in angstrom, charges in e,
with the same constant k_e as the oracle (Eq. solv times 4 pi k_e).

* Born (kappa = 0) and Born-Debye-Hueckel (kappa > 0) for a central charge.
* Kirkwood's series for any charges inside one dielectric sphere.
* Concentric spheres: a per-multipole linear solve that matches the
  potential and eps d phi / d r across every interface (Laplace shells with
  r^n and r^(-n-1), Yukawa shells with i_n(kappa r), k_n(kappa r)).  It
  covers the Stern-layer sphere and a concentric solvent-filled cavity.
"""

from __future__ import annotations

import math

import numpy as np
from scipy.special import eval_legendre, spherical_in, spherical_kn

from .bem import KE


def born(a, eps_in, eps_out, q=1.0):
    """Central charge q in a sphere of radius a, no salt."""
    return 0.5 * KE * q * q * (1.0 / eps_out - 1.0 / eps_in) / a


def born_dh(a, eps_in, eps_out, kappa, q=1.0):
    """Central charge with salt outside (Debye-Hueckel)."""
    return 0.5 * KE * q * q * (1.0 / (eps_out * (1.0 + kappa * a)) - 1.0 / eps_in) / a


def born_dh_dkappa(a, eps_in, eps_out, kappa, q=1.0):
    return -0.5 * KE * q * q / (eps_out * (1.0 + kappa * a) ** 2)


def born_dh_deps_out(a, eps_in, eps_out, kappa, q=1.0):
    return -0.5 * KE * q * q / (eps_out ** 2 * (1.0 + kappa * a) * a)


def stern_central(a, b, eps_in, eps_out, kappa, q=1.0):
    """Central charge; protein radius a (eps_in), Stern shell a<r<b (eps_out,
    no salt), salt solvent r>b (eps_out, kappa)."""
    return 0.5 * KE * q * q * ((1.0 / eps_out - 1.0 / eps_in) / a
                               + (1.0 / (1.0 + kappa * b) - 1.0) / (eps_out * b))


def _log_deriv_k(n, x):
    """x k_n'(x) / k_n(x) for the modified spherical Bessel function k_n."""
    return x * spherical_kn(n, x, derivative=True) / spherical_kn(n, x)


def kirkwood(a, eps_in, eps_out, kappa, xyz, q, tol=1e-15, nmax=400):
    """Kirkwood series energy for point charges inside a sphere of radius a.

    phi_reac(r_j) = sum_k q_k / (4 pi eps_in a) sum_n (r_j r_k / a^2)^n R_n P_n(cos g_jk)
    R_n = (eps_in (n+1) + eps_out g_n) / (eps_in n - eps_out g_n), g_n the log
    derivative x k_n'(x)/k_n(x) at x = kappa a (g_n = -(n+1) when kappa = 0).
    Energy = 1/2 * 4 pi k_e * sum_j q_j phi_reac(r_j).
    """
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    r = np.linalg.norm(xyz, axis=1)
    rr = np.outer(r, r) / (a * a)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosg = (xyz @ xyz.T) / np.outer(r, r)
    cosg = np.where(np.isfinite(cosg), np.clip(cosg, -1.0, 1.0), 1.0)
    qq = np.outer(q, q)
    total = 0.0
    for n in range(nmax):
        g = -(n + 1.0) if kappa == 0.0 else _log_deriv_k(n, kappa * a)
        Rn = (eps_in * (n + 1) + eps_out * g) / (eps_in * n - eps_out * g)
        term = np.sum(qq * rr ** n * eval_legendre(n, cosg)) * Rn
        total += term
        if n > 2 and abs(term) < tol * max(abs(total), 1e-300) and rr.max() ** n < tol:
            break
    # 1/2 * 4 pi k_e * sum q phi, with phi carrying 1/(4 pi eps_in a)
    return 0.5 * KE * total / (eps_in * a)


def kirkwood_phi_reac(a, eps_in, eps_out, kappa, xyz, q, at, nmax=400, tol=1e-15):
    """Reaction potential (in the oracle's units, G with 1/(4 pi)) at points ``at``."""
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    at = np.asarray(at, dtype=np.float64).reshape(-1, 3)
    rk = np.linalg.norm(xyz, axis=1)
    rj = np.linalg.norm(at, axis=1)
    rr = np.outer(rj, rk) / (a * a)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosg = (at @ xyz.T) / np.outer(rj, rk)
    cosg = np.where(np.isfinite(cosg), np.clip(cosg, -1.0, 1.0), 1.0)
    out = np.zeros(len(at))
    for n in range(nmax):
        g = -(n + 1.0) if kappa == 0.0 else _log_deriv_k(n, kappa * a)
        Rn = (eps_in * (n + 1) + eps_out * g) / (eps_in * n - eps_out * g)
        term = (rr ** n * eval_legendre(n, cosg)) @ q * Rn
        out += term
        if n > 2 and rr.max() ** n < tol:
            break
    return out / (4.0 * math.pi * eps_in * a)


def _basis(n, kappa, r, which, rs):
    """Radial solutions and their r-derivatives in one shell.

    Laplace: (r/rs)^n, (r/rs)^(-n-1).  Yukawa: i_n(kappa r), k_n(kappa r).
    """
    if kappa == 0.0:
        if which == 0:
            return (r / rs) ** n, n * (r / rs) ** n / r
        return (r / rs) ** (-n - 1), -(n + 1) * (r / rs) ** (-n - 1) / r
    x = kappa * r
    if which == 0:
        return spherical_in(n, x), kappa * spherical_in(n, x, derivative=True)
    return spherical_kn(n, x), kappa * spherical_kn(n, x, derivative=True)


def concentric(radii, eps, kappa, charge_region, xyz, q, nmax=200, tol=1e-14):
    """Energy of charges in one Laplace layer of nested spheres about the origin.

    ``radii`` ascending (m interfaces); ``eps``, ``kappa`` per layer from the
    innermost ball (0) to the unbounded outer layer (m).  In layer l the
    potential of mode n is A_l f_l + B_l g_l (+ the Coulomb term in the charge
    layer); B_0 = 0 (regular at the origin), A_m = 0 (decay at infinity).
    """
    radii = list(map(float, radii))
    m = len(radii)
    c = int(charge_region)
    if kappa[c] != 0.0:
        raise ValueError("charges must sit in a Laplace layer")
    xyz = np.asarray(xyz, dtype=np.float64).reshape(-1, 3)
    q = np.asarray(q, dtype=np.float64)
    rk = np.linalg.norm(xyz, axis=1)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosg = (xyz @ xyz.T) / np.outer(rk, rk)
    cosg = np.where(np.isfinite(cosg), np.clip(cosg, -1.0, 1.0), 1.0)
    rs = radii[0]
    lo = radii[c - 1] if c > 0 else 0.0
    hi = radii[c] if c < m else math.inf
    if (c > 0 and np.any(rk <= lo)) or np.any(rk >= hi):
        raise ValueError("a charge is outside its layer")
    total = 0.0
    for n in range(nmax):
        # unknowns: A_0, (A_l, B_l) for 0<l<m, B_m  -> 2m unknowns
        cols = [(0, 0)] + [(l, w) for l in range(1, m) for w in (0, 1)] + [(m, 1)]
        col_of = {cw: i for i, cw in enumerate(cols)}
        M = np.zeros((2 * m, 2 * m))
        rhs = np.zeros((2 * m, len(q)))
        for i, a in enumerate(radii):
            for side, l in ((+1, i), (-1, i + 1)):
                for w in (0, 1):
                    if (l, w) not in col_of:
                        continue
                    f, df = _basis(n, kappa[l], a, w, rs)
                    M[2 * i, col_of[(l, w)]] += side * f
                    M[2 * i + 1, col_of[(l, w)]] += side * eps[l] * df
                if l == c:
                    # Coulomb term of a unit-strength charge at radius rk, mode n:
                    # rk^n / r^(n+1) outside the charge radius, r^n / rk^(n+1) inside
                    if a > rk.max():
                        f = rk ** n / a ** (n + 1)
                        df = -(n + 1) * rk ** n / a ** (n + 2)
                    else:
                        f = a ** n / rk ** (n + 1)
                        df = n * a ** (n - 1) / rk ** (n + 1) if n > 0 else 0.0 * rk
                    rhs[2 * i] -= side * f
                    rhs[2 * i + 1] -= side * eps[l] * df
        scale = np.max(np.abs(M), axis=0)
        scale[scale == 0] = 1.0
        sol = np.linalg.solve(M / scale, rhs) / scale[:, None]
        # reaction potential of mode n at charge j from charge k (unit strength)
        with np.errstate(invalid="ignore", divide="ignore"):
            fA = _basis(n, 0.0, rk, 0, rs)[0] if (c, 0) in col_of else 0.0
            fB = _basis(n, 0.0, rk, 1, rs)[0] if (c, 1) in col_of else 0.0
        A = sol[col_of[(c, 0)]] if (c, 0) in col_of else np.zeros(len(q))
        B = sol[col_of[(c, 1)]] if (c, 1) in col_of else np.zeros(len(q))
        # phi_jk = (A_k f(r_j) + B_k g(r_j)) P_n(cos g_jk) / (4 pi eps_c)
        phi = (np.outer(np.atleast_1d(fA), A) + np.outer(np.atleast_1d(fB), B)) \
            * eval_legendre(n, cosg)
        term = q @ phi @ q
        total += term
        if n > 3 and abs(term) < tol * abs(total):
            break
    return 0.5 * KE * total / eps[c]
