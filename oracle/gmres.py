"""Restarted GMRES (oracle, test infrastructure only).

The paper solves the BEM system with a Krylov method and does one operator
evaluation per iteration (sec. 2.3); tolerance from the parameter tables of
sec. 3.  Restart length, start vector and orthogonalisation are not given;
this reading uses x0 = 0, restart m, modified Gram-Schmidt Arnoldi, Givens
rotations, and stops when the implicit residual ||r|| / ||b|| <= tol.
"""

from __future__ import annotations

import numpy as np


def gmres(apply, b, tol=1e-6, restart=100, max_iter=1000, x0=None):
    """Solve A x = b; returns (x, history of implicit relative residuals)."""
    b = np.asarray(b, dtype=np.float64)
    n = len(b)
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    bnorm = np.linalg.norm(b)
    hist = []
    if bnorm == 0.0:
        return np.zeros(n), hist
    total = 0
    while total < max_iter:
        r = b - apply(x) if total > 0 or x0 is not None else b.copy()
        beta = np.linalg.norm(r)
        if beta / bnorm <= tol:
            break
        m = min(restart, max_iter - total)
        V = np.zeros((m + 1, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(m):
            w = apply(V[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0.0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                a, c = H[i, j], H[i + 1, j]
                H[i, j] = cs[i] * a + sn[i] * c
                H[i + 1, j] = -sn[i] * a + cs[i] * c
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            total += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if hist[-1] <= tol or total >= max_iter:
                break
        y = np.zeros(j_done)
        for i in range(j_done - 1, -1, -1):
            y[i] = (g[i] - H[i, i + 1:j_done] @ y[i + 1:j_done]) / H[i, i]
        x = x + V[:j_done].T @ y
        if hist and hist[-1] <= tol:
            break
    return x, hist
