"""GPU parity of the block-diagonal right preconditioner.

* pbtc_precond_apply (M^-1 and M^-T) against the oracle's block inverse on
  the reduced three-region system (every sign and eps ratio of the row
  formula; FP64 self integrals on both sides: 1e-11).
* Solves with precond = block_diag reach the same solution as the oracle's
  LU solve (direct FP64: 1e-8 at tol 1e-11) and the same energy as the
  unpreconditioned GPU solve (FP32-refined treecode: 1e-5), in fewer GMRES
  iterations.
* The adjoint solve (preconditioned with M^-T) gives the oracle's gradients.
* A batch of independent molecules converges system by system.
"""

import numpy as np
import pytest

import synth
from oracle import Oracle
from oracle.adjoint import gradients

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def layered():
    prob = synth.config3_multisurface(nu=8, cav_nu=4, n_charges=200)
    o = Oracle(prob)
    A = o.matrix()
    return prob, o, A, o.rhs()


def test_precond_apply(layered, gpu_lib):
    from paper_1309_4018_amd import lib

    prob, o, A, b = layered
    pl = lib.plan_for(prob, op="direct", precision="fp64")
    pl.setup()
    v = np.random.default_rng(5).normal(size=o.n)
    for tr in (False, True):
        got = pl.precond_apply(v, transpose=tr).cpu().numpy()
        assert _rel(got, o.precond_apply(v, transpose=tr)) < 1e-11


def test_direct_solve_matches_lu(layered, gpu_lib):
    from paper_1309_4018_amd import lib

    prob, o, A, b = layered
    x_lu = np.linalg.solve(A, b)
    iters = {}
    for pc in ("none", "block_diag"):
        pl = lib.plan_for(prob, op="direct", precision="fp64", tol=1e-11, max_iter=3000,
                          precond=pc)
        res = pl.solve()
        assert _rel(pl.solution(), x_lu) < 1e-8
        iters[pc] = res["n_iter"]
    assert iters["block_diag"] < 0.6 * iters["none"]


def test_treecode_fp32_refined_energy(gpu_lib):
    from paper_1309_4018_amd import lib

    prob = synth.config2_star(nu=16, n_charges=300)
    out = {}
    for pc in ("none", "block_diag"):
        pl = lib.plan_for(prob, precision="fp32_refined", tol=1e-6, theta=0.5, P=6, precond=pc)
        res = pl.solve()
        assert res["converged"] == 1 and res["final_rel_res"] <= 1e-6
        out[pc] = res
    e0, e1 = out["none"]["energy_kJmol"], out["block_diag"]["energy_kJmol"]
    assert abs(e1 - e0) < 1e-5 * abs(e0)
    assert out["block_diag"]["n_iter"] < out["none"]["n_iter"]


def test_adjoint_with_precond(gpu_lib):
    from paper_1309_4018_amd import lib

    prob = synth.config1_kirkwood_sphere(nu=8)
    g = gradients(Oracle(prob))
    pl = lib.plan_for(prob, op="direct", precision="fp64", tol=1e-12, precond="block_diag")
    pl.solve()
    dq, dk, de = pl.backward()
    assert _rel(dq, g["dE_dq"]) < 1e-8
    assert abs(dk[1] - g["dE_dkappa"][1]) < 1e-6 * abs(g["dE_dkappa"][1])
    assert _rel(de, g["dE_deps"]) < 1e-8


def test_batch_with_precond(gpu_lib):
    from paper_1309_4018_amd import lib

    probs = [synth.config1_kirkwood_sphere(nu=n, seed=s) for n, s in ((4, 1), (8, 2), (6, 3))]
    bp = lib.batch_problem(probs)
    pl = lib.Plan(bp, lib.default_params(op="direct", precision="fp64", tol=1e-10,
                                         precond="block_diag"), "cuda:0")
    pl.solve()
    e, r, _ = lib.systems(pl)
    assert len(e) == len(probs)
    for k, prob in enumerate(probs):
        e_ref = Oracle(prob).solve(tol=1e-12).energy
        assert abs(e[k] - e_ref) < 1e-8 * abs(e_ref)
        assert r[k] <= 1e-10
