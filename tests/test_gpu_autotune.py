"""GPU check of the autotuner: the chosen (theta, P, ncrit, direct_below)
meets the error budget against the direct FP64 operator, and every measured
candidate's error falls with P at fixed theta."""

import pytest

import synth

pytestmark = pytest.mark.gpu


def test_autotune_meets_budget(gpu_lib):
    from paper_1309_4018_amd import lib
    from paper_1309_4018_amd.autotune import autotune

    prob = lib.Problem.from_synth(synth.config1_kirkwood_sphere())
    best, rows = autotune(prob, budget=1e-4, thetas=(0.4, 0.6), orders=(4, 6),
                          ncrits=(64, 128), direct_belows=(-1,))
    chosen = [r for r in rows if all(r[k] == best[k] for k in best)]
    assert chosen and chosen[0]["err_fp32"] <= 1e-4
    for th in (0.4, 0.6):
        e = {r["P"]: r["err_fp64"] for r in rows if r["theta"] == th and r["ncrit"] == 128}
        assert e[6] < e[4]


def _merged(problems):
    """One synth problem holding several molecules (regions renumbered)."""
    regions, surfaces, charges = [], [], {}
    for p in problems:
        r0 = len(regions)
        regions += [synth.Region(r.eps, r.kappa, r.name) for r in p.regions]
        surfaces += [synth.Surface(s.verts, s.tris, s.inner + r0, s.outer + r0, s.name)
                     for s in p.surfaces]
        for r, (x, q) in p.charges.items():
            charges[r + r0] = (x, q)
    return synth.Problem(regions, surfaces, charges, name="merged")


def test_autotune_batch_choice_meets_budget_against_oracle(gpu_lib):
    """The autotuner on a 5-molecule uneven batch (theta x P grid, then
    ncrit, then the P2P / M2P work tiles): the chosen parameters' FP32
    treecode matvec is within the error budget of the dense FP64 oracle's
    matrix (Eq. matrix of every molecule; the oracle is independent of the
    library's direct operator the tuner measures against)."""
    import numpy as np

    from oracle import Oracle
    from paper_1309_4018_amd import lib
    from paper_1309_4018_amd.autotune import autotune

    mols = synth.config4_batch(n_mol=5, nu_cap=6)
    budget = 1e-4
    best, rows = autotune(lib.batch_problem(mols), budget=budget, thetas=(0.4, 0.6),
                          orders=(4, 6), ncrits=(64, 128), unit_sources=(512, 1024),
                          unit_cells=(32, 64))
    assert any(r["unit_sources"] == 512 for r in rows)  # the tile stage ran
    o = Oracle(_merged(mols))
    A = o.matrix()
    x = np.random.default_rng(4).normal(size=o.n)
    ref = A @ x
    pl = lib.Plan(lib.batch_problem(mols), lib.default_params(**best))
    pl.setup()
    y = pl.matvec(x, lib.FP32).cpu().numpy()
    assert np.max(np.abs(y - ref)) / np.max(np.abs(ref)) <= budget
