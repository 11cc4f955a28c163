#!/usr/bin/env python3
"""Benchmark of the treecode BEM hot path on one MI355X.

One step is one pass of the whole path on the star-shaped protein-like
surface (40,500 panels, K = 4 -> 162,000 Gauss points, 2,000 charges,
eps 4/80, kappa 0.125, theta 0.5, P 6): device set-up (panel geometry, Gauss
points, Morton sort, octree, interaction lists, near-singular tables,
Coulomb right-hand side) from inputs resident in HBM, the FP32-bulk GMRES
solve with FP64 iterative refinement to ||b - A x|| / ||b|| <= 1e-5, the
reaction potential and the FP64 energy sum.  The paper's solver is plain
GMRES; the same solve with the block-diagonal right preconditioner is
reported beside it.

value = dense-equivalent interactions per second over the whole step:
(sum over regions of targets x Gauss points) x operator evaluations / step
time.  The JSON line also reports the solve and set-up seconds, the plain FP64
GPU treecode for comparison, matvec-only rates, the P2P/M2P roofline of the
dominant kernel (HIP events on the launch stream, recorded by the library)
and the CPU oracle timed on a bounded sample of rows.  After the timed steps
the adjoint gradient evaluation (dE/dq, dE/dkappa, dE/deps) is timed too.

Other workloads (--workload): sphere (2,048 panels), multisurface (protein,
Stern layer and two cavities, 167,936 panels) and batch (64 independent
star-shaped molecules, 614,420 panels, solved together); --autotune picks
theta, P and the tree parameters first.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32, published (counts packed FP32)
PEAK_FP32_NONPACKED_TFLOPS = 78.6  # one FP32 FMA per lane per cycle: 256 CU x 64 x 2 x 2.4 GHz
PEAK_FP64_TFLOPS = 78.6


def workload(name):
    """(problem, description): a ``synth`` problem, or a list of them (batch)."""
    import synth

    if name == "star":
        return synth.config2_star(), "star-shaped surface 40,500 panels (ico nu=45), 2,000 charges"
    if name == "sphere":
        return synth.config1_kirkwood_sphere(), "Kirkwood sphere 2,048 panels, 9 charges"
    if name == "multisurface":
        return synth.config3_multisurface(), ("protein + Stern + 2 cavities, 167,936 panels, "
                                              "4,000 charges")
    if name == "batch":
        probs = synth.config4_batch(n_mol=64)
        return probs, (f"64 star-shaped molecules, {sum(p.n_panels for p in probs):,} panels, "
                       f"{sum(p.n_charges for p in probs):,} charges, one launch sequence")
    raise SystemExit(f"unknown workload {name}")


def counted_traffic(workload_name, kernel):
    """HBM bytes per launch of ``kernel`` from the committed rocprofv3 counter
    summary of this workload (FETCH_SIZE and WRITE_SIZE scaled by the copy
    probe), or None when there is none or the kernel sources changed since."""
    path = os.path.join(ROOT, "profiles", f"hbm_counters_{workload_name}.txt")
    if not os.path.exists(path):
        return None
    sha, sources, traffic = None, [], {}
    for line in open(path):
        if line.startswith("source_sha256:"):
            sha = line.split(":", 1)[1].strip()
        elif line.startswith("sources:"):
            sources = line.split(":", 1)[1].split()
        elif line.startswith("kernel "):
            parts = line.split()
            traffic[parts[1]] = float(parts[parts.index("traffic_bytes") + 1])
    if not sha or not sources or kernel not in traffic:
        return None
    h = hashlib.sha256()
    for f in sources:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return traffic[kernel] if h.hexdigest() == sha else None


def make_plan(lib, prob, **params):
    if isinstance(prob, list):
        return lib.Plan(lib.batch_problem(prob), lib.default_params(**params), "cuda:0")
    return lib.plan_for(prob, "cuda:0", **params)


def cpu_baseline(prob, seconds=15.0):
    """Oracle (dense FP64, numpy) on a bounded sample of operator rows."""
    from oracle import Oracle

    o = Oracle(prob)
    rng = np.random.default_rng(0)
    x = rng.normal(size=o.n)
    t = 0
    rows_done = 0
    inter = 0.0
    start = time.perf_counter()
    batch = 8
    n_t = o.ns[t]
    src_per_row = sum(o.ns[s] * o.par.k for r in o.row_regions(t) for s in o.bound[r])
    while time.perf_counter() - start < seconds:
        rows = rng.choice(n_t, size=batch, replace=False)
        o.apply_rows(x, t, rows)
        rows_done += batch
        inter += batch * src_per_row
    el = time.perf_counter() - start
    return {"value": inter / el, "unit": "interactions/s", "cores": 1, "kind": "oracle",
            "sample": f"{rows_done} collocation points x both row blocks (all {src_per_row} "
                      f"Gauss-point interactions per point, dense FP64 numpy), {el:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="star")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="also run one elementwise copy of this size (HBM counter calibration)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose theta, P, ncrit, direct_below with the autotuner first")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="adjoint (gradient) evaluations timed after the solves")
    ap.add_argument("--minimal", action="store_true",
                    help="only the timed FP32-refined steps (for counter collection)")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU: the multi-GPU path (targets sharded across GPUs, "
              "unknown vector all-gathered per matvec) is designed but not built.",
              file=sys.stderr)
        return 2

    import torch

    from paper_1309_4018_amd import lib

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    if a.copy_probe_mb > 0:
        n = int(a.copy_probe_mb * 2 ** 20 / 4)
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        torch.mul(src, 1.0, out=dst)  # reads n*4 bytes, writes n*4 bytes
        torch.cuda.synchronize(dev)
        del src, dst
    prob, desc = workload(a.workload)
    probs = prob if isinstance(prob, list) else [prob]
    n_panels = sum(p.n_panels for p in probs)
    n_charges = sum(p.n_charges for p in probs)
    tree = {"theta": 0.5, "P": 6}
    tune = None
    if a.autotune:
        from paper_1309_4018_amd.autotune import autotune

        t = time.perf_counter()
        tree, rows = autotune(lib.batch_problem(probs), budget=1e-4,
                              base={"precision": "fp32_refined", "tol": 1e-5})
        tune = {"seconds": time.perf_counter() - t, "chosen": tree, "candidates": len(rows)}
    # kernel timing on every 8th FP32 operator evaluation (each timed launch
    # costs an event pair on the stream)
    pl = make_plan(lib, prob, precision="fp32_refined", tol=1e-5, profile=8, **tree)
    pl.setup()
    for _ in range(a.warmup):
        pl.solve(force_setup=True)
    torch.cuda.synchronize(dev)
    results = []
    t0 = time.perf_counter()
    for _ in range(a.steps):
        results.append(pl.solve(force_setup=True))
    torch.cuda.synchronize(dev)
    el = time.perf_counter() - t0
    ms = 1e3 * el / a.steps
    last = results[-1]
    dense = last["n_dense_equiv"]
    nmv = sum(r["n_matvec_fp32"] + r["n_matvec_fp64"] for r in results)
    value = dense * nmv / el

    # roofline of the dominant kernel over the timed steps: the library times
    # each P2P, Laplace M2P and Yukawa M2P launch of the FP32 operator with
    # HIP events on the launch stream
    def tot(key):
        return sum(r[key] for r in results)

    kern = {
        "p2p": (tot("t_p2p_s"), tot("n_p2p_launch"), tot("p2p_flop")),
        "m2p_laplace": (tot("t_m2p_s") - tot("t_m2p_yuk_s"),
                        tot("n_m2p_launch") - tot("n_m2p_yuk_launch"),
                        tot("m2p_flop") - tot("m2p_yuk_flop")),
        "m2p_yukawa": (tot("t_m2p_yuk_s"), tot("n_m2p_yuk_launch"), tot("m2p_yuk_flop")),
    }
    name = max(kern, key=lambda k: kern[k][0])
    t_k, n_k, f_k = kern[name]
    achieved = f_k / t_k / 1e12 if t_k > 0 else 0.0
    roofline = {"bound": "alu", "kernel": name, "achieved": achieved, "peak": PEAK_FP32_TFLOPS,
                "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_TFLOPS,
                "traffic": counted_traffic(a.workload, name),
                "avg_launch_ms": 1e3 * t_k / max(n_k, 1),
                "flop_per_launch": f_k / max(n_k, 1),
                "peak_nonpacked_fp32": PEAK_FP32_NONPACKED_TFLOPS,
                "kernels": {k: {"tflops": (v[2] / v[0] / 1e12) if v[0] else 0.0,
                                "avg_launch_ms": 1e3 * v[0] / max(v[1], 1),
                                "timed_launches": v[1]} for k, v in kern.items()}}

    if a.minimal:
        print(json.dumps({"metric": "BEM matvec interactions/s + GMRES solve s to 1e-5; "
                                    "FP32-bulk vs FP64", "value": value,
                          "unit": "interactions/s", "n_gpus": 1, "steps": a.steps,
                          "warmup": a.warmup, "ms_per_step": ms, "roofline": roofline,
                          "minimal": True}))
        return 0

    # matvec-only rates (FP32 and FP64 operators) with events on the stream
    x = torch.randn(pl.n_unknowns, dtype=torch.float64, device=dev)
    mv = {}
    for name, prec in (("fp32", lib.FP32), ("fp64", lib.FP64)):
        for _ in range(2):
            pl.matvec(x, prec)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        reps = 10
        s.record()
        for _ in range(reps):
            pl.matvec(x, prec)
        e.record()
        torch.cuda.synchronize(dev)
        mv[name] = s.elapsed_time(e) / 1e3 / reps

    # plain FP64 GPU treecode, same accuracy target
    # adjoint: dE/dq, dE/dkappa, dE/deps after the last solve
    adjoint = None
    if a.adjoint > 0:
        pl.backward()  # builds the transposed operator
        torch.cuda.synchronize(dev)
        t = time.perf_counter()
        for _ in range(a.adjoint):
            dq32, _, _ = pl.backward()
        torch.cuda.synchronize(dev)
        adjoint = {"seconds": (time.perf_counter() - t) / a.adjoint,
                   "gmres_iterations": pl.last.n_iter,
                   "matvecs_fp32": pl.last.n_matvec_fp32, "matvecs_fp64": pl.last.n_matvec_fp64}

    pl64 = make_plan(lib, prob, precision="fp64", tol=1e-5, **tree)
    pl64.setup()
    r64 = [pl64.solve(force_setup=True) for _ in range(max(a.fp64_steps, 1))]
    solve64 = float(np.median([r["t_solve_s"] for r in r64]))
    solve32 = float(np.median([r["t_solve_s"] for r in results]))
    if adjoint is not None:
        pl64.backward()
        torch.cuda.synchronize(dev)
        t = time.perf_counter()
        for _ in range(a.adjoint):
            dq64, _, _ = pl64.backward()
        torch.cuda.synchronize(dev)
        adjoint["fp64_seconds"] = (time.perf_counter() - t) / a.adjoint
        adjoint["fp64_gmres_iterations"] = pl64.last.n_iter
        adjoint["speedup_vs_fp64"] = adjoint["fp64_seconds"] / adjoint["seconds"]
        adjoint["dE_dq_rel_diff_vs_fp64"] = float(np.max(np.abs(dq32 - dq64)) / np.max(np.abs(dq64)))

    # the same solve with the block-diagonal right preconditioner (not in the
    # paper; reported beside the headline, which follows the paper's solver)
    plp = make_plan(lib, prob, precision="fp32_refined", tol=1e-5, precond="block_diag", **tree)
    plp.setup()
    rp = [plp.solve(force_setup=True) for _ in range(max(a.fp64_steps, 1))]
    precond = {"solve_s": float(np.median([r["t_solve_s"] for r in rp])),
               "gmres_iterations": rp[-1]["n_iter"],
               "matvecs_fp32": rp[-1]["n_matvec_fp32"], "matvecs_fp64": rp[-1]["n_matvec_fp64"],
               "energy_kJmol": rp[-1]["energy_kJmol"], "final_rel_res": rp[-1]["final_rel_res"]}
    del plp

    out = {
        "metric": "BEM matvec interactions/s + GMRES solve s to 1e-5; FP32-bulk vs FP64",
        "value": value,
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operator, f64 krylov/refinement",
        "data": "synthetic",
        "config": {"workload": desc, "panels": int(n_panels),
                   "gauss_points": int(n_panels * 4), "charges": int(n_charges),
                   "K": 4, "theta": tree["theta"], "P": tree["P"], "tol": 1e-5,
                   "precision": "fp32 bulk, fp64 refinement"},
        "solve_s": solve32,
        "setup_s": float(np.median([r["t_setup_s"] for r in results])),
        "setup_phase_s": dict(zip(
            ["sort", "octree", "lists", "near_columns", "host_tables", "near_values_precond_rhs"],
            np.median([r["t_setup_phase_s"] for r in results], axis=0).tolist())),
        "energy_kJmol": last["energy_kJmol"],
        "final_rel_res": last["final_rel_res"],
        "gmres_iterations": last["n_iter"],
        "matvecs_fp32": last["n_matvec_fp32"], "matvecs_fp64": last["n_matvec_fp64"],
        "dense_interactions_per_matvec": dense,
        "p2p_pairs_per_matvec": last["n_p2p_pairs"],
        "m2p_evals_per_matvec": last["n_m2p_evals"],
        "near_entries": last["n_near_entries"],
        "matvec_s": mv,
        "matvec_interactions_per_s": {k: dense / v for k, v in mv.items()},
        "fp64_solve_s": solve64,
        "fp64_energy_kJmol": r64[-1]["energy_kJmol"],
        "fp64_iterations": r64[-1]["n_iter"],
        "speedup_fp32_refined_vs_fp64": solve64 / solve32 if solve32 else None,
        "block_diag_precond": precond,
        "adjoint": adjoint,
        "autotune": tune,
        "roofline": roofline,
    }
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(probs[0], a.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
