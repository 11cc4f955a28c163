"""GPU parity of the multi-surface system at full size: protein surface and
Stern layer at 81,920 panels each, two cavities at 2,048 (167,936 panels,
335,872 unknowns, 4,000 charges), in the launch configuration the benchmark
times (treecode, theta = 0.5, P = 6, FP32 bulk with FP64 refinement, all
surface-pair blocks of all regions in shared launches).

The oracle cannot assemble this system; it evaluates sampled rows one by one
(Eq. matrix in its multi-surface form, sec. 2.2):
* rows of A x for a random x, 48 per surface, both row halves (the surface
  seen from its inner and from its outer region), FP64 and FP32 operators;
* the residual b - A x of the GPU solution on those rows;
* the reaction potential (Eq. reac_integral) at 24 sampled charges.
Tolerance 3e-4 of each row block's scale (Taylor truncation at P = 6,
theta = 0.5).  The FP32-refined energy agrees with the plain FP64 treecode's
to 1e-4 at the benchmark's tolerance and to 1e-6 when both solve to 1e-8.
"""

import numpy as np
import pytest

import synth
from oracle import Oracle
from oracle.integrals import green

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def c3():
    prob = synth.config3_multisurface()
    return prob, Oracle(prob)


@pytest.fixture(scope="module")
def plan(c3, gpu_lib):
    from paper_1309_4018_amd import lib

    pl = lib.plan_for(c3[0], precision="fp32_refined", tol=1e-5, theta=0.5, P=6)
    pl.setup()
    return pl


def _rows(o, rng):
    return [rng.choice(n, size=min(48, n), replace=False) for n in o.ns]


def test_matvec_sampled_rows_every_surface(c3, plan):
    from paper_1309_4018_amd import lib

    prob, o = c3
    rng = np.random.default_rng(31)
    x = rng.normal(size=o.n)
    rows = _rows(o, rng)
    refs = [o.apply_rows(x, t, rows[t]) for t in range(len(o.ns))]
    for prec in (lib.FP64, lib.FP32):
        y = plan.matvec(x, prec).cpu().numpy()
        for t, nt in enumerate(o.ns):
            for half in range(2):
                got = y[o.uoff[t] + half * nt + rows[t]]
                ref = refs[t][half]
                assert np.max(np.abs(got - ref)) < 3e-4 * np.max(np.abs(ref)), (prec, t, half)


def test_solution_residual_and_reaction_potential(c3, plan):
    prob, o = c3
    res = plan.solve()
    assert res["converged"] == 1 and res["final_rel_res"] <= 1e-5
    x = plan.solution()
    rng = np.random.default_rng(32)
    rows = _rows(o, rng)
    pairs = []
    for t, nt in enumerate(o.ns):
        Ax = o.apply_rows(x, t, rows[t])
        X = o.pan[t].centre[rows[t]]
        for half, r in enumerate(o.row_regions(t)):
            sel = o.qreg == r
            b = np.zeros(len(rows[t]))
            if np.any(sel):
                R = np.linalg.norm(X[:, None, :] - o.qx[sel][None, :, :], axis=2)
                b = green(R, o.kappa[r]) @ o.q[sel] / o.eps[r]
            pairs.append(((t, half), Ax[half], b))
    # rows of charge-free regions have b = 0: one scale, the largest |b|
    scale = max(np.max(np.abs(b)) for _, _, b in pairs)
    for key, ax, b in pairs:
        assert np.max(np.abs(ax - b)) < 3e-4 * scale, key
    # reaction potential at sampled charges, all in the protein region
    ks = rng.choice(len(o.q), size=24, replace=False)
    phi_ref = np.zeros(len(ks))
    r = 0
    for s in o.bound[r]:
        V, K = o.point_blocks(o.qx[ks], s, o.kappa[r])
        ns = o.ns[s]
        phi_s, psi_s = x[o.uoff[s]:o.uoff[s] + ns], x[o.uoff[s] + ns:o.uoff[s] + 2 * ns]
        phi_ref += o.sigma(r, s) * (o.ratio(r, s) * (V @ psi_s) - K @ phi_s)
    phi = plan.phi_reac()[ks]
    assert np.max(np.abs(phi - phi_ref)) < 3e-4 * np.max(np.abs(phi_ref))
    # the energy is the reduction of the reaction potential (Eq. solv)
    e = 0.5 * 4 * np.pi * 1389.35458 * float(o.q @ plan.phi_reac())
    assert abs(e - res["energy_kJmol"]) < 1e-12 * abs(e)


def test_energy_fp32_refined_vs_fp64(c3, plan):
    """At the benchmark's tolerance (1e-5) the FP32-refined energy is within
    1e-4 of the plain FP64 treecode's; with both solved to 1e-8 the two differ
    only by the FP32 rounding that refinement removes (1e-6)."""
    from paper_1309_4018_amd import lib

    e32 = plan.solve()["energy_kJmol"]
    p64 = lib.plan_for(c3[0], precision="fp64", tol=1e-8, theta=0.5, P=6, max_iter=3000)
    e64 = p64.solve()["energy_kJmol"]
    assert abs(e32 - e64) < 1e-4 * abs(e64)
    p32 = lib.plan_for(c3[0], precision="fp32_refined", tol=1e-8, theta=0.5, P=6, max_iter=3000)
    e32t = p32.solve()["energy_kJmol"]
    assert abs(e32t - e64) < 1e-6 * abs(e64)
