"""Exact discrete gradients of the solvation energy (oracle; test only).

With the discrete system A x = B q (Eq. matrix; B maps the charges to the
Coulomb right-hand side of Eq. matel) and dG = 1/2 C q^T S x (Eq. solv;
S maps the unknowns to phi_reac at the charges, Eq. reac_integral;
C = 4 pi k_e), the adjoint lambda solves A^T lambda = S^T q and
    d dG / d q       = 1/2 C (S x + B^T lambda)
    d dG / d p       = 1/2 C [q^T (dS/dp) x - lambda^T (dA/dp) x + lambda^T (dB/dp) q]
for p = kappa_r or eps_r.  kappa enters through the Yukawa kernels
(d G_Y / d kappa = -exp(-kappa R)/(4 pi),
 d (n.grad G_Y) / d kappa = -kappa n.(x-y) exp(-kappa R)/(4 pi R))
and the semi-analytic self term; eps enters through the ratios c_rs and the
1/eps_r of the Coulomb term.
"""

from __future__ import annotations

import math

import numpy as np

from .bem import KE

C_ENERGY = 4.0 * math.pi * KE


def gradients(oracle, x=None):
    """Returns dict with energy, dE_dq (n_q,), dE_dkappa and dE_deps per region."""
    o = oracle
    A = o.matrix()
    B = o.coulomb_matrix()
    S = o.reaction_matrix()
    q = o.q
    if x is None:
        x = np.linalg.solve(A, B @ q)
    lam = np.linalg.solve(A.T, S.T @ q)
    out = {"x": x, "lam": lam, "energy": 0.5 * C_ENERGY * float(q @ (S @ x))}
    out["dE_dq"] = 0.5 * C_ENERGY * (S @ x + B.T @ lam)
    nreg = len(o.eps)
    dk = np.zeros(nreg)
    de = np.zeros(nreg)
    for r in range(nreg):
        dA = o.dmatrix_dkappa(r)
        dB = o.coulomb_matrix(dkappa_region=r)
        dS = o.reaction_matrix(
            coef=lambda rr, s: (o.sigma(rr, s) * o.ratio(rr, s), -o.sigma(rr, s)),
            kind="dkappa", only_region=r)
        dk[r] = 0.5 * C_ENERGY * (q @ (dS @ x) - lam @ (dA @ x) + lam @ (dB @ q))
        dAe = o.dmatrix_deps(r)
        # B carries 1/eps_row: d/d eps_r scales the rows of region r by -1/eps_r
        dBe = np.zeros_like(B)
        for t in range(len(o.ns)):
            nt = o.ns[t]
            for half, rr in enumerate(o.row_regions(t)):
                if rr == r:
                    r0 = o.uoff[t] + half * nt
                    dBe[r0:r0 + nt] = -B[r0:r0 + nt] / o.eps[r]
        dSe = o.reaction_matrix(coef=lambda rr, s: (o.sigma(rr, s) * o.dratio(rr, s, r), 0.0))
        de[r] = 0.5 * C_ENERGY * (q @ (dSe @ x) - lam @ (dAe @ x) + lam @ (dBe @ q))
    out["dE_dkappa"] = dk
    out["dE_deps"] = de
    return out
