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
