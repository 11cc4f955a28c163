"""Dense-direct boundary-element Poisson-Boltzmann solver (oracle).

Test infrastructure only: the product library never imports, links or calls
anything here.  This is the plain, slow, obviously correct FP64 reference the
GPU path is checked against.

Formulation
-----------
Single surface (sec. 2.1 Eq. nBEM, sec. 2.2 Eqs. nBEM_disc, matrix, matel):
    [ 1/2 I + K_L    -V_L          ] [phi ]   [Q]
    [ 1/2 I - K_Y    (e1/e2) V_Y   ] [dphi] = [0]
with G carrying 1/(4 pi) (Eq. nBEM) and the ratio e1/e2 in front of V_Y as in
the discrete equations (the continuous equation prints e2/e1; substituting
flux continuity of Eq. pde into the exterior identity gives e1/e2).

Several surfaces (sec. 2.2, multi-surface problems): the paper defers the
formulation to Altman et al.; the reading used here is Green's third
identity written in every region.  Surface s separates its inner region I(s)
from its outer region O(s), its normal points from I(s) into O(s), and its
unknowns are phi_s and psi_s = d phi / d n on the inner side; flux
continuity gives the outer-side derivative (eps_I(s) / eps_O(s)) psi_s.
Region r is bounded by B(r) = {s : I(s) = r or O(s) = r}; with
sigma_rs = +1 if I(s) = r else -1 and c_rs = 1 if I(s) = r else
eps_I(s) / eps_r, the row block of surface t seen from region
r in {I(t), O(t)} reads
    1/2 phi_t(x_i) - sum_{s in B(r)} sigma_rs [c_rs V_r^{ts} psi_s - K_r^{ts} phi_s](x_i)
        = sum_{k in r} q_k / eps_r G_r(x_i, x_k).
For one surface this is exactly Eq. matrix.

Reaction potential and energy (Eqs. reac_integral, solv): for a charge at
x_k in region r,
    phi_reac(x_k) = sum_{s in B(r)} sigma_rs [c_rs V_r psi_s - K_r phi_s](x_k),
    dG_solv = 1/2 * 4 pi k_e * sum_k q_k phi_reac(x_k)   [kJ/mol],
k_e = e^2 N_A / (4 pi eps_0 * 1 A) = 1389.35458 kJ A / (mol e^2); the 4 pi
undoes the 1/(4 pi) inside G.

Unknown order: for each surface s in input order, [phi_s (n_s), psi_s (n_s)].
Row order: for each surface t, [rows seen from I(t), rows seen from O(t)].
"""

from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from .geometry import panels
from .gmres import gmres
from .integrals import green, panel_integrals, self_integral

KE = 1389.35458  # kJ * A / (mol * e^2)
ENERGY_FACTOR = 0.5 * 4.0 * math.pi * KE


@dataclass
class Params:
    k: int = 4
    k_fine: int = 19
    nk: int = 5
    thres: float = 2.0
    tol: float = 1e-6
    restart: int = 100
    max_iter: int = 1000


class Oracle:
    """Dense FP64 BEM for a ``synth.Problem``-like object.

    The problem needs ``regions`` (eps, kappa), ``surfaces`` (verts, tris,
    inner, outer) and ``charges`` {region: (xyz, q)}.
    """

    def __init__(self, problem, params: Params | None = None):
        self.prob = problem
        self.par = params or Params()
        self.eps = np.array([r.eps for r in problem.regions], dtype=np.float64)
        self.kappa = np.array([r.kappa for r in problem.regions], dtype=np.float64)
        self.pan = [panels(s.verts, s.tris) for s in problem.surfaces]
        self.ns = [p.n for p in self.pan]
        self.uoff = np.concatenate([[0], np.cumsum([2 * n for n in self.ns])])
        self.n = int(self.uoff[-1])
        self.inner = [s.inner for s in problem.surfaces]
        self.outer = [s.outer for s in problem.surfaces]
        nreg = len(problem.regions)
        self.bound = [[s for s in range(len(self.ns)) if r in (self.inner[s], self.outer[s])]
                      for r in range(nreg)]
        self.qx, self.q, self.qreg = problem.all_charges()
        self._cache = {}

    # -- region graph --------------------------------------------------------
    def sigma(self, r, s):
        return 1.0 if self.inner[s] == r else -1.0

    def ratio(self, r, s, eps=None):
        eps = self.eps if eps is None else eps
        return 1.0 if self.inner[s] == r else eps[self.inner[s]] / eps[r]

    def row_regions(self, t):
        return (self.inner[t], self.outer[t])

    # -- blocks ---------------------------------------------------------------
    def block(self, t, s, kappa, kind="value", rows=None):
        """V_r^{ts}, K_r^{ts} for collocation points of t (optionally a subset)."""
        pt = self.pan[t]
        idx = np.arange(pt.n) if rows is None else np.asarray(rows)
        X = pt.centre[idx]
        self_idx = idx if s == t else None
        P = self.par
        return panel_integrals(X, self.pan[s], kappa, P.k, P.k_fine, P.thres, P.nk,
                               self_idx=self_idx, kind=kind)

    def point_blocks(self, X, s, kappa, kind="value"):
        """V, K for arbitrary points (charges); no self panel."""
        P = self.par
        return panel_integrals(X, self.pan[s], kappa, P.k, P.k_fine, P.thres, P.nk,
                               self_idx=None, kind=kind)

    def _assemble(self, coef, kind="value", identity=True, only_region=None, kappa=None):
        """Sum over row blocks of coef(r, s) = (a_V, a_K) times V_r^{ts}, K_r^{ts}."""
        kap = self.kappa if kappa is None else np.asarray(kappa, dtype=np.float64)
        A = np.zeros((self.n, self.n))
        for t in range(len(self.ns)):
            nt = self.ns[t]
            for half, r in enumerate(self.row_regions(t)):
                r0 = self.uoff[t] + half * nt
                if identity:
                    A[r0:r0 + nt, self.uoff[t]:self.uoff[t] + nt] += 0.5 * np.eye(nt)
                if only_region is not None and r != only_region:
                    continue
                for s in self.bound[r]:
                    aV, aK = coef(r, s)
                    if aV == 0.0 and aK == 0.0:
                        continue
                    key = (t, s, float(kap[r]), kind)
                    if key not in self._cache:
                        self._cache[key] = self.block(t, s, kap[r], kind)
                    V, K = self._cache[key]
                    ns = self.ns[s]
                    A[r0:r0 + nt, self.uoff[s] + ns:self.uoff[s] + 2 * ns] += aV * V
                    A[r0:r0 + nt, self.uoff[s]:self.uoff[s] + ns] += aK * K
        return A

    def matrix(self, eps=None, kappa=None):
        """Dense system matrix A (n, n)."""
        eps = self.eps if eps is None else np.asarray(eps, dtype=np.float64)
        return self._assemble(
            lambda r, s: (-self.sigma(r, s) * self.ratio(r, s, eps), self.sigma(r, s)),
            kappa=kappa)

    def dratio(self, r, s, p):
        """d c_rs / d eps_p."""
        i = self.inner[s]
        if i == r:
            return 0.0
        return (1.0 if p == i else 0.0) / self.eps[r] - (
            self.eps[i] / self.eps[r] ** 2 if p == r else 0.0)

    def dmatrix_deps(self, p):
        """d A / d eps_p (only the c_rs ratios depend on eps)."""
        return self._assemble(lambda r, s: (-self.sigma(r, s) * self.dratio(r, s, p), 0.0),
                              identity=False)

    def dmatrix_dkappa(self, r0):
        """d A / d kappa_r0 (rows seen from region r0, derivative kernels)."""
        return self._assemble(
            lambda r, s: (-self.sigma(r, s) * self.ratio(r, s), self.sigma(r, s)),
            kind="dkappa", identity=False, only_region=r0)

    def apply_rows(self, x, t, rows):
        """Rows ``rows`` of both row blocks of surface t applied to x
        (matrix-free; for parity checks at sizes too large to assemble)."""
        rows = np.asarray(rows)
        out = []
        for half, r in enumerate(self.row_regions(t)):
            y = 0.5 * x[self.uoff[t] + rows]
            for s in self.bound[r]:
                V, K = self.block(t, s, self.kappa[r], rows=rows)
                ns = self.ns[s]
                phi = x[self.uoff[s]:self.uoff[s] + ns]
                psi = x[self.uoff[s] + ns:self.uoff[s] + 2 * ns]
                y = y - self.sigma(r, s) * (self.ratio(r, s) * (V @ psi) - K @ phi)
            out.append(y)
        return out

    def coulomb_matrix(self, eps=None, kappa=None, dkappa_region=None):
        """B (n, n_q): right-hand side = B q (point evaluation, no quadrature)."""
        eps = self.eps if eps is None else np.asarray(eps, dtype=np.float64)
        kap = self.kappa if kappa is None else np.asarray(kappa, dtype=np.float64)
        B = np.zeros((self.n, len(self.q)))
        for t in range(len(self.ns)):
            nt = self.ns[t]
            X = self.pan[t].centre
            for half, r in enumerate(self.row_regions(t)):
                cols = np.nonzero(self.qreg == r)[0]
                if len(cols) == 0:
                    continue
                if dkappa_region is not None and r != dkappa_region:
                    continue
                R = np.linalg.norm(X[:, None, :] - self.qx[cols][None, :, :], axis=2)
                if dkappa_region is None:
                    g = green(R, kap[r])
                else:
                    g = -np.exp(-kap[r] * R) / (4.0 * math.pi)
                r0 = self.uoff[t] + half * nt
                B[r0:r0 + nt, cols] = g / eps[r]
        return B

    def rhs(self):
        return self.coulomb_matrix() @ self.q

    def reaction_matrix(self, coef=None, kind="value", only_region=None):
        """S (n_q, n): phi_reac at the charges = S x.

        ``coef(r, s)`` = (a_V, a_K) defaults to (sigma_rs c_rs, -sigma_rs);
        ``kind`` = "dkappa" with ``only_region`` gives d S / d kappa_r.
        """
        if coef is None:
            coef = lambda r, s: (self.sigma(r, s) * self.ratio(r, s), -self.sigma(r, s))
        S = np.zeros((len(self.q), self.n))
        for r in np.unique(self.qreg):
            if only_region is not None and r != only_region:
                continue
            rows = np.nonzero(self.qreg == r)[0]
            for s in self.bound[r]:
                aV, aK = coef(r, s)
                if aV == 0.0 and aK == 0.0:
                    continue
                key = ("q", int(r), s, float(self.kappa[r]), kind)
                if key not in self._cache:
                    self._cache[key] = self.point_blocks(self.qx[rows], s, self.kappa[r], kind)
                V, K = self._cache[key]
                ns = self.ns[s]
                S[np.ix_(rows, np.arange(self.uoff[s] + ns, self.uoff[s] + 2 * ns))] += aV * V
                S[np.ix_(rows, np.arange(self.uoff[s], self.uoff[s] + ns))] += aK * K
        return S

    # -- block-diagonal preconditioner (the paper names none) ----------------
    def block_diagonal(self):
        """(np_total, 2, 2) diagonal blocks of A, surfaces in order.

        For panel p of surface t: rows (t, I(t)) and (t, O(t)) of its own
        collocation point, columns phi_p and psi_p.  From the row formula:
        entry (r, phi) = 1/2 + sigma_rt K_r(p, p) and (r, psi) =
        -sigma_rt c_rt V_r(p, p), with K_r(p, p) = 0 (flat panel, centre in
        its plane) and V_r(p, p) the semi-analytic self integral.
        """
        out = []
        for t, nt in enumerate(self.ns):
            M = np.zeros((nt, 2, 2))
            for half, r in enumerate(self.row_regions(t)):
                V = self_integral(self.pan[t], np.arange(nt), self.kappa[r], self.par.nk)
                M[:, half, 0] = 0.5
                M[:, half, 1] = -self.sigma(r, t) * self.ratio(r, t) * V
            out.append(M)
        return np.concatenate(out)

    def precond_apply(self, v, transpose=False):
        """M^-1 v (or M^-T v) for the block-diagonal M; v in the unknown layout."""
        inv = np.linalg.inv(self.block_diagonal())
        if transpose:
            inv = np.transpose(inv, (0, 2, 1))
        v = np.asarray(v, dtype=np.float64)
        y = np.empty_like(v)
        p0 = 0
        for t, nt in enumerate(self.ns):
            i0 = self.uoff[t] + np.arange(nt)
            i1 = i0 + nt
            blk = inv[p0:p0 + nt]
            y[i0] = blk[:, 0, 0] * v[i0] + blk[:, 0, 1] * v[i1]
            y[i1] = blk[:, 1, 0] * v[i0] + blk[:, 1, 1] * v[i1]
            p0 += nt
        return y

    # -- solve ----------------------------------------------------------------
    def solve(self, tol=None, restart=None, max_iter=None, use_lu=False):
        P = self.par
        A = self.matrix()
        b = self.rhs()
        if use_lu:
            x = np.linalg.solve(A, b)
            hist = []
        else:
            x, hist = gmres(lambda v: A @ v, b, tol or P.tol, restart or P.restart,
                            max_iter or P.max_iter)
        S = self.reaction_matrix()
        phi_reac = S @ x
        energy = ENERGY_FACTOR * float(self.q @ phi_reac)
        return Solution(x=x, history=hist, phi_reac=phi_reac, energy=energy, A=A, b=b, S=S,
                        oracle=self)

    def split(self, x):
        """Per surface (phi_s, psi_s) views of an unknown vector."""
        out = []
        for s, ns in enumerate(self.ns):
            o = self.uoff[s]
            out.append((x[o:o + ns], x[o + ns:o + 2 * ns]))
        return out


@dataclass
class Solution:
    x: np.ndarray
    history: list
    phi_reac: np.ndarray
    energy: float
    A: np.ndarray
    b: np.ndarray
    S: np.ndarray
    oracle: Oracle

    @property
    def n_iter(self):
        return len(self.history)
