"""Pins of the oracle's block-diagonal preconditioner (CPU).

The paper solves with unpreconditioned GMRES (sec. 2.3); the block-diagonal
right preconditioner is an addition, so what fixes it is algebra, not a
printed value:
* its blocks are the 2 x 2 diagonal blocks of the dense system matrix, which
  the oracle assembles through its general panel-integral path (self rule
  chosen by index there, taken directly here);
* right preconditioning leaves the solution unchanged: GMRES on A M^-1
  followed by x = M^-1 y reaches the LU solution of A x = b (and of the
  transposed system with M^-T);
* it lowers the iteration count on the multi-surface system.
"""

import numpy as np
import pytest

import synth
from oracle import Oracle
from oracle.gmres import gmres


def _diag_blocks(o, A):
    out = []
    for t, nt in enumerate(o.ns):
        u = o.uoff[t]
        for i in range(nt):
            idx = [u + i, u + nt + i]
            out.append(A[np.ix_(idx, idx)])
    return np.array(out)


@pytest.fixture(scope="module")
def layered():
    # protein / Stern / solvent with a cavity (kappa > 0 outside): every
    # sign and ratio of the row formula appears
    prob = synth.config3_multisurface(nu=4, cav_nu=2, n_charges=20)
    o = Oracle(prob)
    return o, o.matrix(), o.rhs()


def test_blocks_equal_matrix_diagonal(layered):
    o, A, _ = layered
    M = o.block_diagonal()
    assert M.shape == (sum(o.ns), 2, 2)
    np.testing.assert_allclose(M, _diag_blocks(o, A), rtol=1e-13, atol=1e-15)


def test_blocks_single_sphere():
    o = Oracle(synth.config1_kirkwood_sphere(nu=4))
    np.testing.assert_allclose(o.block_diagonal(), _diag_blocks(o, o.matrix()), rtol=1e-13,
                               atol=1e-15)


def test_apply_is_block_inverse(layered):
    o, A, _ = layered
    v = np.random.default_rng(1).normal(size=o.n)
    D = np.zeros_like(A)
    for t, nt in enumerate(o.ns):
        u = o.uoff[t]
        for i in range(nt):
            idx = [u + i, u + nt + i]
            D[np.ix_(idx, idx)] = A[np.ix_(idx, idx)]
    np.testing.assert_allclose(D @ o.precond_apply(v), v, rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(D.T @ o.precond_apply(v, transpose=True), v, rtol=1e-12,
                               atol=1e-12)


def test_right_preconditioned_solution_unchanged(layered):
    o, A, b = layered
    x_lu = np.linalg.solve(A, b)
    y, hist_p = gmres(lambda v: A @ o.precond_apply(v), b, tol=1e-11, restart=100,
                      max_iter=2000)
    x = o.precond_apply(y)
    assert np.linalg.norm(b - A @ x) / np.linalg.norm(b) < 1e-10
    assert np.max(np.abs(x - x_lu)) < 1e-7 * np.max(np.abs(x_lu))
    _, hist = gmres(lambda v: A @ v, b, tol=1e-5, restart=100, max_iter=2000)
    _, hist_p5 = gmres(lambda v: A @ o.precond_apply(v), b, tol=1e-5, restart=100,
                       max_iter=2000)
    assert len(hist_p5) < len(hist)


def test_transposed_system(layered):
    o, A, _ = layered
    c = np.random.default_rng(2).normal(size=o.n)
    lam_lu = np.linalg.solve(A.T, c)
    y, _ = gmres(lambda v: A.T @ o.precond_apply(v, transpose=True), c, tol=1e-11, restart=100,
                 max_iter=2000)
    lam = o.precond_apply(y, transpose=True)
    assert np.max(np.abs(lam - lam_lu)) < 1e-7 * np.max(np.abs(lam_lu))
