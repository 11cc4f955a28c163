"""GPU parity for multi-surface problems (protein + Stern layer + cavities).

A reduced version of the three-region system (protein and Stern surfaces at
ico nu = 8, cavities at oct nu = 4: 2,816 panels, 5,632 unknowns, 200
charges) is small enough for the dense oracle.  It exercises every block
type: surface pairs seen from two Laplace regions, Laplace + Yukawa,
cross-surface near-singular panels (Stern layer 2 A from the protein
surface) and charges bounded by three surfaces.  Tolerances as for the
sphere: 1e-12 direct FP64, 2e-5 direct FP32, Taylor truncation for the
treecode; energies 1e-9 (direct FP64 solve) and 1e-4 (FP32-refined
treecode).  Concentric cavity / Stern spheres check the GPU energy against
the oracle on problems whose oracle is itself pinned to a closed form.
"""

import numpy as np
import pytest

import synth
from oracle import Oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def small():
    prob = synth.config3_multisurface(nu=8, cav_nu=4, n_charges=200)
    o = Oracle(prob)
    sol = o.solve(tol=1e-12)
    rng = np.random.default_rng(21)
    x = rng.normal(size=o.n) * np.abs(sol.x).mean()
    return prob, o, sol, x, sol.A @ x


def _rel(a, b):
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def test_rhs_and_direct_matvec(small, gpu_lib):
    from paper_1309_4018_amd import lib

    prob, o, sol, x, y = small
    pl = lib.plan_for(prob, op="direct", precision="fp64")
    pl.setup()
    assert _rel(pl.rhs().cpu().numpy(), sol.b) < 1e-13
    assert _rel(pl.matvec(x, lib.FP64).cpu().numpy(), y) < 1e-12
    assert _rel(pl.matvec(x, lib.FP32).cpu().numpy(), y) < 2e-5


def test_treecode_matvec(small, gpu_lib):
    from paper_1309_4018_amd import lib

    prob, o, sol, x, y = small
    errs = []
    for P in (4, 6, 8):
        pl = lib.plan_for(prob, theta=0.5, P=P, ncrit=64)
        pl.setup()
        errs.append(_rel(pl.matvec(x, lib.FP64).cpu().numpy(), y))
    assert errs[1] < 3e-4 and errs[2] < errs[1] < errs[0]


def test_solves_match_oracle(small, gpu_lib):
    from paper_1309_4018_amd import lib

    prob, o, sol, x, y = small
    pd = lib.plan_for(prob, op="direct", precision="fp64", tol=1e-12)
    r = pd.solve()
    assert r["converged"] == 1
    assert abs(r["energy_kJmol"] - sol.energy) < 1e-9 * abs(sol.energy)
    assert _rel(pd.solution(), sol.x) < 1e-8
    assert _rel(pd.phi_reac(), sol.phi_reac) < 1e-8
    pt = lib.plan_for(prob, precision="fp32_refined", tol=1e-6, theta=0.5, P=6)
    r = pt.solve()
    assert r["converged"] == 1 and r["final_rel_res"] <= 1e-6
    assert abs(r["energy_kJmol"] - sol.energy) < 1e-4 * abs(sol.energy)


@pytest.mark.parametrize("case", ["stern", "cavity", "ioncavity"])
def test_concentric_spheres(gpu_lib, case):
    from paper_1309_4018_amd import lib

    xq = np.array([[0.0, 0.0, 2.8], [0.8, 2.0, -1.6], [-2.4, 0.8, 0.8]])
    qq = np.array([1.0, -0.5, 0.7])
    if case == "stern":
        radii, eps, kap, creg, xc = [4.0, 6.0], [4, 80, 80], [0, 0, 0.125], 0, xq
    elif case == "cavity":
        radii, eps, kap, creg, xc = [2.0, 6.0], [80, 4, 80], [0, 0, 0.125], 1, xq * 1.25
    else:  # ions inside a cavity with its own Stern layer
        radii, eps, kap = [2.5, 4.0, 9.0, 11.0], [80, 80, 4, 80, 80], [0.125, 0, 0, 0, 0.125]
        creg, xc = 2, xq * 2.3
    p = synth.concentric_spheres(radii, eps, kap, (xc, qq), creg, nu=8)
    ref = Oracle(p).solve(tol=1e-12).energy
    pl = lib.plan_for(p, precision="fp32_refined", tol=1e-7, theta=0.5, P=8)
    r = pl.solve()
    assert abs(r["energy_kJmol"] - ref) < 1e-4 * abs(ref)


def test_ion_holding_cavity_protein(gpu_lib):
    """Star protein, Stern layer, a solvent cavity and an ion-holding cavity
    with its own Stern shell (six regions, five surfaces): GPU direct FP64
    and FP32-refined treecode against the dense oracle."""
    from paper_1309_4018_amd import lib

    prob = synth.ion_cavity_protein(nu=8, cav_nu=4, n_charges=100)
    o = Oracle(prob)
    sol = o.solve(tol=1e-12)
    x = np.random.default_rng(9).normal(size=o.n)
    pd = lib.plan_for(prob, op="direct", precision="fp64", tol=1e-12, max_iter=4000)
    pd.setup()
    assert _rel(pd.matvec(x, lib.FP64).cpu().numpy(), sol.A @ x) < 1e-12
    rd = pd.solve()
    assert abs(rd["energy_kJmol"] - sol.energy) < 1e-9 * abs(sol.energy)
    pt = lib.plan_for(prob, precision="fp32_refined", tol=1e-7, theta=0.5, P=8, max_iter=4000)
    rt = pt.solve()
    assert abs(rt["energy_kJmol"] - sol.energy) < 1e-4 * abs(sol.energy)
