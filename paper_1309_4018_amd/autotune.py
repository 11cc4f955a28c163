"""Autotuner for the treecode parameters.

Three kinds of parameters are chosen, in this order:
* accuracy: the MAC parameter theta and the expansion order P (sec. 2.3,
  Eqs. multexp and MAC) -- they change the answer; every candidate of the
  grid is measured at the default speed parameters;
* the octree cell size ncrit (speed; rounding and truncation move only
  marginally);
* the work tiles of the P2P and M2P kernels: sources per P2P work unit and
  far cells per M2P work unit (speed only: the same sums in another order of
  units), starting from the library's automatic choice.  The target-group size is not tuned: it is the wavefront width
  (64), which keeps every list a wave walks wave-uniform (scalar loads of
  sources and moments); a smaller group would leave lanes idle.

For every candidate the operator error is measured against the library's own
direct FP64 operator (every pair by the K-point rule plus the same near-field
corrections: the discrete operator the treecode approximates) on one random
vector, as max_i |y_i - y_i^direct| / max_i |y_i^direct|.  Among the
(theta, P) candidates within ``budget`` the fastest FP32 matvec (HIP-event
time on the current stream, median of a few repetitions) wins; each speed
stage then keeps a candidate only if it is faster and still within the
budget.  Every evaluation runs in the HIP kernels of libpbtc; this module
only orchestrates and times.
"""

from __future__ import annotations

import itertools

import numpy as np

from . import lib


def _time_matvec(plan, x, precision, reps=5):
    import torch

    for _ in range(2):
        plan.matvec(x, precision)
    times = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        plan.matvec(x, precision)
        e.record()
        torch.cuda.synchronize()
        times.append(s.elapsed_time(e) / 1e3)
    return float(np.median(times))


SPEED_KEYS = ("ncrit", "direct_below", "unit_sources", "unit_cells")


def autotune(problem, budget=1e-4, thetas=(0.4, 0.5, 0.6), orders=(4, 6, 8),
             ncrits=(64, 128, 256), direct_belows=(-1,), unit_sources=(512, 1024, 2048),
             unit_cells=(32, 64, 128), device="cuda:0", seed=0, base=None):
    """Returns (best parameter dict, list of measured candidates).

    ``problem`` is a ``lib.Problem``; ``base`` extra parameters passed to
    every plan (tolerance, precision...).
    """
    import torch

    base = dict(base or {})
    ref_plan = lib.Plan(problem, lib.default_params(**dict(base, op="direct",
                                                           precision="fp64")), device)
    ref_plan.setup()
    rng = np.random.default_rng(seed)
    x = torch.as_tensor(rng.normal(size=ref_plan.n_unknowns), dtype=torch.float64,
                        device=device)
    y_ref = ref_plan.matvec(x, lib.FP64)
    scale = float(y_ref.abs().max())
    del ref_plan
    rows = []

    def measure(theta, P, speed):
        pl = lib.Plan(problem, lib.default_params(**dict(base, theta=theta, P=P, **speed)),
                      device)
        pl.setup()
        err64 = float((pl.matvec(x, lib.FP64) - y_ref).abs().max()) / scale
        err32 = float((pl.matvec(x, lib.FP32) - y_ref).abs().max()) / scale
        t32 = _time_matvec(pl, x, lib.FP32)
        row = dict(theta=theta, P=P, err_fp64=err64, err_fp32=err32, matvec_s_fp32=t32, **speed)
        rows.append(row)
        return row

    # tiles start automatic (0: chosen by the library from the lists' sizes)
    speed = {"ncrit": ncrits[len(ncrits) // 2], "direct_below": direct_belows[0],
             "unit_sources": 0, "unit_cells": 0}
    first = [measure(t, p, speed) for t, p in itertools.product(thetas, orders)]
    ok = [r for r in first if r["err_fp32"] <= budget]
    if not ok:
        ok = [min(first, key=lambda r: r["err_fp32"])]
    best = min(ok, key=lambda r: r["matvec_s_fp32"])

    def stage(cands):
        nonlocal best
        for c in cands:
            sp = {k: best[k] for k in SPEED_KEYS}
            sp.update(c)
            if all(sp[k] == best[k] for k in SPEED_KEYS):
                continue
            r = measure(best["theta"], best["P"], sp)
            if (r["err_fp32"] <= max(budget, best["err_fp32"])
                    and r["matvec_s_fp32"] < best["matvec_s_fp32"]):
                best = r

    stage([{"ncrit": nc, "direct_below": db} for nc, db in itertools.product(ncrits, direct_belows)])
    stage([{"unit_sources": us, "unit_cells": uc}
           for us, uc in itertools.product(unit_sources, unit_cells)])
    params = {k: best[k] for k in ("theta", "P") + SPEED_KEYS}
    return params, rows
