"""GPU parity of the full uneven batch: 64 star-shaped molecules (1,280 to
32,000 panels, 614,420 in all, 28,089 charges) solved together in shared
launches (treecode, theta = 0.5, P = 6, FP32 bulk with FP64 refinement),
both as one multi-system problem and through pbtc_solve_batch.

* Every molecule of at most 5,120 panels (30 of them): its energy against
  the dense FP64 oracle's LU solve of that molecule (stored by
  tests/golden/make_c4_energies.py), 1e-4 relative.
* Every larger molecule: the residual b - A x of its part of the GPU
  solution on 16 sampled rows of each row half, against the oracle's rows
  (3e-4 of the row scale).
"""

import json
import os

import numpy as np
import pytest

import synth
from oracle import Oracle
from oracle.integrals import green

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden", "c4_energies.json")
PRM = dict(precision="fp32_refined", tol=1e-5, theta=0.5, P=6)


@pytest.fixture(scope="module")
def mols():
    return synth.config4_batch(n_mol=64)


@pytest.fixture(scope="module")
def solved(mols, gpu_lib):
    from paper_1309_4018_amd import lib

    pl = lib.Plan(lib.batch_problem(mols), lib.default_params(**PRM))
    res = pl.solve()
    e, rel, first = lib.systems(pl)
    return pl, res, e, rel, first


def test_small_molecules_energy_vs_dense_oracle(mols, solved):
    pl, res, e, rel, first = solved
    assert res["converged"] == 1 and len(e) == len(mols)
    assert np.all(rel <= 1e-5)
    gold = json.load(open(GOLD))
    assert len(gold["molecules"]) == 30
    for m in gold["molecules"]:
        i = m["index"]
        assert mols[i].n_panels == m["panels"]
        assert abs(e[i] - m["energy_kJmol"]) < 1e-4 * abs(m["energy_kJmol"]), i


def test_large_molecules_sampled_residual(mols, solved):
    pl, res, e, rel, first = solved
    x = pl.solution()
    rng = np.random.default_rng(41)
    for i, m in enumerate(mols):
        if m.n_panels <= 5120:
            continue
        o = Oracle(m)
        xi = x[first[i]:first[i] + o.n]
        rows = rng.choice(o.ns[0], size=16, replace=False)
        Ax = o.apply_rows(xi, 0, rows)
        X = o.pan[0].centre[rows]
        R = np.linalg.norm(X[:, None, :] - o.qx[None, :, :], axis=2)
        b0 = green(R, 0.0) @ o.q / o.eps[0]
        scale = np.max(np.abs(b0))
        assert np.max(np.abs(Ax[0] - b0)) < 3e-4 * scale, i
        assert np.max(np.abs(Ax[1])) < 3e-4 * scale, i


def test_solve_batch_entry_point_matches(mols, solved, gpu_lib):
    """pbtc_solve_batch over 64 single-molecule plans gives the same energies."""
    from paper_1309_4018_amd import lib

    pl, res, e, rel, first = solved
    plans = [lib.plan_for(m, **PRM) for m in mols]
    out = lib.Batch(plans).solve()
    got = np.array([r["energy_kJmol"] for r in out])
    assert np.all([r["converged"] == 1 for r in out])
    assert np.max(np.abs(got - e) / np.abs(e)) < 1e-9
