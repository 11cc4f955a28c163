"""Allocation-free Coulomb energy (pbtc_coulomb_energy_noalloc) against the
workspace entry point pbtc_coulomb_energy, through the C interface: two calls
in a row on one GPU, the second with a smaller input (fewer charges, fewer
systems), each equal to the workspace entry point's result (same FP64
kernels: bit for bit)."""

import ctypes as C

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu


def _both(lib, pl):
    n = C.c_int()
    lib.check(pl.lib.pbtc_get_systems(pl.h, C.byref(n), None, None, None), pl.h)
    out = []
    for fn in (pl.lib.pbtc_coulomb_energy, pl.lib.pbtc_coulomb_energy_noalloc):
        tot = C.c_double()
        per = np.full(n.value, np.nan)
        lib.check(fn(pl.h, C.c_void_p(pl.ws.data_ptr()), pl.stream, C.byref(tot),
                     C.c_void_p(per.ctypes.data)), pl.h)
        out.append((tot.value, per))
    return out


def test_noalloc_coulomb_matches_workspace_entry_point(gpu_lib):
    from paper_1309_4018_amd import lib

    big = lib.Plan(lib.batch_problem(synth.config4_batch(n_mol=6, nu_cap=8)),
                   lib.default_params(op="direct", precision="fp64"))
    small = lib.plan_for(synth.config1_kirkwood_sphere(nu=4), op="direct", precision="fp64")
    for pl in (big, small):
        pl.setup()
        (t_ws, per_ws), (t_na, per_na) = _both(lib, pl)
        assert np.isfinite(t_ws) and t_ws != 0.0
        assert t_na == t_ws
        assert np.array_equal(per_na, per_ws)
    assert len(per_ws) == 1  # the second (smaller) input: one system
