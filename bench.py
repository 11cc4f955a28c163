#!/usr/bin/env python3
"""Benchmark of the treecode BEM hot path on one MI355X.

Headline (the JSON line's value): one step is one pass of the whole path on
the star-shaped protein-like surface (40,500 panels, K = 4 -> 162,000 Gauss
points, 2,000 charges, eps 4/80, kappa 0.125, theta 0.5, P 6): device
set-up (panel geometry, Gauss points, Morton sort, octree, interaction
lists, near-singular tables, Coulomb right-hand side) from inputs resident
in HBM, the FP32-bulk GMRES solve with FP64 iterative refinement to
||b - A x|| / ||b|| <= 1e-5, the reaction potential and the FP64 energy.
value = dense-equivalent interactions per second over the whole step:
(sum over regions of targets x Gauss points) x operator evaluations / step
time.

The same line carries, per configuration, the timed figures of the
other workloads (``configs``): the Kirkwood sphere (2,048 panels, dense
direct FP64, the plain method), the multi-surface system (protein, Stern
layer, two cavities: 167,936 panels) with its adjoint gradient (dE/dq,
dE/dkappa, dE/deps), and the uneven batch of 64 molecules (614,420 panels)
with theta and P chosen by the autotuner over {0.4, 0.5, 0.6} x {4, 6, 8}.
Each reports set-up and solve seconds for the FP32-refined and the plain
FP64 treecode, matvec rates, executed P2P pairs and M2P evaluations per
second, kernel launches per operator evaluation (one launch graph) and the
roofline of every P2P / M2P kernel, forward and transposed (HIP events on
the launch stream, recorded by the library).  cpu_baseline: the CPU oracle
(dense FP64 NumPy) on worker processes over the host's cores, on a bounded
sample of operator rows of the star workload, plus one full oracle solve of
the Kirkwood sphere.
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

METRIC = "BEM matvec interactions/s + GMRES solve s to 1e-5; FP32-bulk vs FP64"
PEAK_FP32_TFLOPS = 157.3  # MI355X vector FP32, published (counts packed FP32)
PEAK_FP64_TFLOPS = 78.6
KINDS = ["p2p", "m2p_laplace", "m2p_yukawa", "adj_p2p", "adj_m2p_laplace", "adj_m2p_yukawa",
         "m2p_laplace_yukawa"]
KERNEL_NAMES = {"p2p": "k_p2p", "m2p_laplace": "k_m2p<float, P, 0, -1>",
                "m2p_yukawa": "k_m2p<float, P, 1, -1>", "adj_p2p": "k_adj_p2p",
                "adj_m2p_laplace": "k_adj_m2p<float, P, 0>",
                "adj_m2p_yukawa": "k_adj_m2p<float, P, 1>",
                "m2p_laplace_yukawa": "k_m2p<float, P, 0, 1> (and <1, 1> for two Yukawa kernels)"}


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
                       f"{sum(p.n_charges for p in probs):,} charges, one launch graph")
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


def kernel_rooflines(results, kinds=range(7)):
    """Per kernel kind: algorithmic TFLOP/s over the timed launches, average
    launch duration and fractions of the FP32 peaks."""
    out = {}
    for k in kinds:
        t = sum(r["t_kernel_s"][k] for r in results)
        n = sum(r["n_kernel_launch"][k] for r in results)
        f = sum(r["kernel_flop"][k] for r in results)
        if n == 0 or t <= 0:
            continue
        tf = f / t / 1e12
        out[KINDS[k]] = {"kernel": KERNEL_NAMES[KINDS[k]], "bound": "alu", "achieved": tf,
                         "peak": PEAK_FP32_TFLOPS, "unit": "TFLOP/s", "frac": tf / PEAK_FP32_TFLOPS,
                         "avg_launch_ms": 1e3 * t / n, "flop_per_launch": f / n,
                         "timed_launches": n}
    return out


def time_matvecs(torch, lib, pl, reps=10):
    dev = pl.device
    x = torch.randn(pl.n_unknowns, dtype=torch.float64, device=dev)
    out = {}
    for name, prec in (("fp32", lib.FP32), ("fp64", lib.FP64)):
        for _ in range(2):
            pl.matvec(x, prec)
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(reps):
            pl.matvec(x, prec)
        e.record()
        torch.cuda.synchronize(dev)
        out[name] = s.elapsed_time(e) / 1e3 / reps
    return out


def run_config(torch, lib, prob, tree, steps, warmup, fp64_steps, adjoint, precond=True,
               eager_compare=True, profile=8):
    """Timed figures of one workload (see the module docstring)."""
    dev = torch.device("cuda:0")
    pl = make_plan(lib, prob, precision="fp32_refined", tol=1e-5, profile=profile, **tree)
    pl.setup()
    for _ in range(warmup):
        pl.solve(force_setup=True)
    torch.cuda.synchronize(dev)
    results = []
    t0 = time.perf_counter()
    for _ in range(steps):
        results.append(pl.solve(force_setup=True))
    torch.cuda.synchronize(dev)
    el = time.perf_counter() - t0
    last = results[-1]
    dense = last["n_dense_equiv"]
    nmv = sum(r["n_matvec_fp32"] + r["n_matvec_fp64"] for r in results)
    out = {
        "ms_per_step": 1e3 * el / steps,
        "steps": steps,
        "dense_interactions_per_s": dense * nmv / el,
        "setup_s": float(np.median([r["t_setup_s"] for r in results])),
        "solve_s": float(np.median([r["t_solve_s"] for r in results])),
        "energy_kJmol": last["energy_kJmol"],
        "final_rel_res": last["final_rel_res"],
        "converged": last["converged"],
        "gmres_iterations": last["n_iter"],
        "matvecs_fp32": last["n_matvec_fp32"], "matvecs_fp64": last["n_matvec_fp64"],
        "dense_interactions_per_matvec": dense,
        "p2p_pairs_per_matvec": last["n_p2p_pairs"],
        "m2p_evals_per_matvec": last["n_m2p_evals"],
        "near_entries": last["n_near_entries"],
        "kernels_per_matvec": last["op_kernels"],
        "work_tiles": {"p2p_sources": last["tile_sources"], "m2p_cells": last["tile_cells"]},
        "graph_launches_per_solve": last["op_graph_launches"],
        "setup_phase_s": dict(zip(
            ["sort", "octree", "lists", "near_columns", "host_tables", "near_values_precond_rhs"],
            np.median([r["t_setup_phase_s"] for r in results], axis=0).tolist())),
    }
    mv = time_matvecs(torch, lib, pl)
    out["matvec_s"] = mv
    out["matvec_dense_interactions_per_s"] = {k: dense / v for k, v in mv.items()}
    out["p2p_pairs_per_s_fp32"] = last["n_p2p_pairs"] / mv["fp32"]
    out["m2p_evals_per_s_fp32"] = last["n_m2p_evals"] / mv["fp32"]
    if eager_compare:
        pe = make_plan(lib, prob, precision="fp32_refined", tol=1e-5, op_graph=0, **tree)
        pe.setup()
        out["matvec_s_kernel_by_kernel"] = time_matvecs(torch, lib, pe)
        pe.solve()
        re_ = pe.solve()
        out["solve_s_kernel_by_kernel"] = re_["t_solve_s"]
        del pe
    adj = None
    if adjoint > 0:
        pl.backward()  # builds the transposed operator
        torch.cuda.synchronize(dev)
        t = time.perf_counter()
        ares = []
        for _ in range(adjoint):
            dq32, dk32, de32 = pl.backward()
            ares.append(pl.last.as_dict())
        torch.cuda.synchronize(dev)
        adj = {"seconds": (time.perf_counter() - t) / adjoint,
               "gmres_iterations": pl.last.n_iter,
               "matvecs_fp32": pl.last.n_matvec_fp32, "matvecs_fp64": pl.last.n_matvec_fp64}
        out["adjoint"] = adj
    rl = kernel_rooflines(results, (0, 1, 2, 6))
    if adjoint > 0:
        rl.update(kernel_rooflines(ares, (3, 4, 5)))
    out["rooflines"] = rl

    pl64 = make_plan(lib, prob, precision="fp64", tol=1e-5, **tree)
    pl64.setup()
    r64 = [pl64.solve(force_setup=True) for _ in range(max(fp64_steps, 1))]
    out["fp64_solve_s"] = float(np.median([r["t_solve_s"] for r in r64]))
    out["fp64_setup_s"] = float(np.median([r["t_setup_s"] for r in r64]))
    out["fp64_energy_kJmol"] = r64[-1]["energy_kJmol"]
    out["fp64_iterations"] = r64[-1]["n_iter"]
    out["speedup_fp32_refined_vs_fp64"] = out["fp64_solve_s"] / out["solve_s"]
    out["energy_rel_diff_fp32_refined_vs_fp64"] = abs(
        out["energy_kJmol"] - out["fp64_energy_kJmol"]) / abs(out["fp64_energy_kJmol"])
    if adjoint > 0:
        pl64.backward()
        torch.cuda.synchronize(dev)
        t = time.perf_counter()
        for _ in range(adjoint):
            dq64, dk64, de64 = pl64.backward()
        torch.cuda.synchronize(dev)
        adj["fp64_seconds"] = (time.perf_counter() - t) / adjoint
        adj["fp64_gmres_iterations"] = pl64.last.n_iter
        adj["speedup_vs_fp64"] = adj["fp64_seconds"] / adj["seconds"]
        adj["dE_dq_rel_diff_vs_fp64"] = float(np.max(np.abs(dq32 - dq64)) / np.max(np.abs(dq64)))
        adj["dE_dkappa"] = [float(v) for v in dk32]
        adj["dE_deps"] = [float(v) for v in de32]
    del pl64
    if precond:
        plp = make_plan(lib, prob, precision="fp32_refined", tol=1e-5, precond="block_diag", **tree)
        plp.setup()
        rp = [plp.solve(force_setup=True) for _ in range(max(fp64_steps, 1))]
        out["block_diag_precond"] = {
            "solve_s": float(np.median([r["t_solve_s"] for r in rp])),
            "gmres_iterations": rp[-1]["n_iter"], "energy_kJmol": rp[-1]["energy_kJmol"],
            "final_rel_res": rp[-1]["final_rel_res"]}
        del plp
    return out, results, pl


def _oracle_rows_worker(args):
    """Worker process: oracle rows of the star workload for a fixed time."""
    seconds, seed = args
    sys.path.insert(0, ROOT)
    import synth
    from oracle import Oracle

    o = Oracle(synth.config2_star())
    rng = np.random.default_rng(seed)
    x = np.random.default_rng(0).normal(size=o.n)
    src_per_row = sum(o.ns[s] * o.par.k for r in o.row_regions(0) for s in o.bound[r])
    rows, inter = 0, 0.0
    start = time.perf_counter()
    while time.perf_counter() - start < seconds:
        rr = rng.choice(o.ns[0], size=8, replace=False)
        o.apply_rows(x, 0, rr)
        rows += 8
        inter += 8 * src_per_row
    return rows, inter, time.perf_counter() - start


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(seconds=12.0):
    """The oracle (dense FP64 NumPy, as it stands) on the host: operator rows
    of the star workload in worker processes over the cores (at most 16),
    plus one full solve (assembly + GMRES) of the Kirkwood sphere."""
    import concurrent.futures as cf
    import multiprocessing as mp

    import synth
    from oracle import Oracle
    from oracle import closed_forms as cfm

    ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu))
    t = time.perf_counter()
    with cf.ProcessPoolExecutor(workers, mp_context=mp.get_context("spawn")) as ex:
        parts = list(ex.map(_oracle_rows_worker, [(seconds, 100 + i) for i in range(workers)]))
    wall = time.perf_counter() - t
    rows = sum(p[0] for p in parts)
    inter = sum(p[1] for p in parts)
    busy = max(p[2] for p in parts)
    c1 = synth.config1_kirkwood_sphere()
    t = time.perf_counter()
    sol = Oracle(c1).solve(tol=1e-6)
    c1_s = time.perf_counter() - t
    x, q = c1.charges[0]
    kirk = cfm.kirkwood(4.0, 4.0, 80.0, 0.125, x, q)
    return {"value": inter / busy, "unit": "interactions/s", "cores": workers, "kind": "oracle",
            "sample": (f"{rows} collocation points of the star workload x both row blocks (all "
                       f"Gauss-point interactions per point, dense FP64 NumPy) on {workers} "
                       f"worker processes for {busy:.1f} s ({wall:.1f} s with start-up)"),
            "nproc": ncpu, "cpu_model": cpu_model(),
            "sphere_full_solve": {"seconds": c1_s, "energy_kJmol": sol.energy,
                                  "gmres_iterations": sol.n_iter,
                                  "kirkwood_kJmol": kirk,
                                  "rel_diff_vs_kirkwood": abs(sol.energy - kirk) / abs(kirk),
                                  "what": "Oracle(config1).solve(tol=1e-6): dense assembly of "
                                          "4,096 x 4,096 A, GMRES, energy"}}


def sphere_config(torch, lib):
    """Kirkwood sphere, the plain method: dense direct FP64 operator and GMRES
    to 1e-6 on the GPU, against Kirkwood's series."""
    import synth
    from oracle import closed_forms as cfm

    prob = synth.config1_kirkwood_sphere()
    pl = lib.plan_for(prob, "cuda:0", op="direct", precision="fp64", tol=1e-6)
    pl.setup()
    pl.solve(force_setup=True)
    torch.cuda.synchronize()
    t = time.perf_counter()
    steps = 5
    for _ in range(steps):
        r = pl.solve(force_setup=True)
    torch.cuda.synchronize()
    el = (time.perf_counter() - t) / steps
    x, q = prob.charges[0]
    kirk = cfm.kirkwood(4.0, 4.0, 80.0, 0.125, x, q)
    mv = time_matvecs(torch, lib, pl)
    return {"ms_per_step": 1e3 * el, "setup_s": r["t_setup_s"], "solve_s": r["t_solve_s"],
            "gmres_iterations": r["n_iter"], "energy_kJmol": r["energy_kJmol"],
            "kirkwood_kJmol": kirk,
            "rel_diff_vs_kirkwood": abs(r["energy_kJmol"] - kirk) / abs(kirk),
            "dense_interactions_per_matvec": r["n_dense_equiv"],
            "matvec_s_fp64": mv["fp64"],
            "matvec_dense_interactions_per_s_fp64": r["n_dense_equiv"] / mv["fp64"],
            "config": "direct FP64 operator (every pair by the K-point rule), GMRES 1e-6"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="star")
    ap.add_argument("--fp64-steps", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--quick", action="store_true", help="headline workload only")
    ap.add_argument("--copy-probe-mb", type=float, default=0.0,
                    help="also run one elementwise copy of this size (HBM counter calibration)")
    ap.add_argument("--autotune", action="store_true",
                    help="choose theta, P, ncrit, direct_below with the autotuner first")
    ap.add_argument("--adjoint", type=int, default=1,
                    help="adjoint (gradient) evaluations timed after the solves")
    ap.add_argument("--minimal", action="store_true",
                    help="only the timed FP32-refined steps (for counter collection)")
    ap.add_argument("--profile-every", type=int, default=16,
                    help="kernel timing on every n-th FP32 operator evaluation (1: every "
                         "evaluation launches kernel by kernel with the moment pass first)")
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

    if a.minimal:
        pl = make_plan(lib, prob, precision="fp32_refined", tol=1e-5, profile=a.profile_every,
                       **tree)
        pl.setup()
        for _ in range(a.warmup):
            pl.solve(force_setup=True)
        torch.cuda.synchronize(dev)
        t0 = time.perf_counter()
        res = [pl.solve(force_setup=True) for _ in range(a.steps)]
        torch.cuda.synchronize(dev)
        el = time.perf_counter() - t0
        nmv = sum(r["n_matvec_fp32"] + r["n_matvec_fp64"] for r in res)
        print(json.dumps({"metric": METRIC, "value": res[-1]["n_dense_equiv"] * nmv / el,
                          "unit": "interactions/s", "n_gpus": 1, "steps": a.steps,
                          "warmup": a.warmup, "ms_per_step": 1e3 * el / a.steps,
                          "rooflines": kernel_rooflines(res, (0, 1, 2, 6)), "minimal": True}))
        return 0

    head, results, pl = run_config(torch, lib, prob, tree, a.steps, a.warmup, a.fp64_steps,
                                   a.adjoint, profile=a.profile_every)
    del pl
    rl = head["rooflines"]
    fwd = {k: v for k, v in rl.items() if not k.startswith("adj")}
    dom = max(fwd, key=lambda k: fwd[k]["avg_launch_ms"] * fwd[k]["timed_launches"])
    roofline = dict(rl[dom])
    roofline["kernel_kind"] = dom
    roofline["traffic"] = counted_traffic(a.workload, dom)
    roofline["traffic_source"] = (f"profiles/hbm_counters_{a.workload}.txt (rocprofv3 FETCH_SIZE "
                                  "and WRITE_SIZE per launch, copy-probe calibrated; null when "
                                  "the kernel sources changed since)")

    configs = {}
    if not a.quick and a.workload == "star":
        configs["sphere_2048_direct_fp64"] = sphere_config(torch, lib)
        p3, d3 = workload("multisurface")
        c3, _, _ = run_config(torch, lib, p3, {"theta": 0.5, "P": 6}, 3, 1, 1, 1)
        c3["workload"] = d3 + " (the adjoint entry is the gradient of this system)"
        configs["multisurface_167936"] = c3
        del p3
        p4, d4 = workload("batch")
        from paper_1309_4018_amd.autotune import autotune

        t = time.perf_counter()
        tree4, rows4 = autotune(lib.batch_problem(p4), budget=1e-4,
                                base={"precision": "fp32_refined", "tol": 1e-5},
                                ncrits=(64, 128, 256), direct_belows=(-1,))
        tune4 = {"seconds": time.perf_counter() - t, "chosen": tree4, "budget": 1e-4,
                 "grid": ("theta {0.4, 0.5, 0.6} x P {4, 6, 8}, then ncrit {64, 128, 256}, "
                          "then P2P tile {512, 1024, 2048} sources x M2P tile {32, 64, 128} cells "
                          "(from the automatic tiles)"),
                 "candidates": [{k: r[k] for k in ("theta", "P", "ncrit", "unit_sources",
                                                   "unit_cells", "err_fp32", "matvec_s_fp32")}
                                for r in rows4]}
        c4, _, _ = run_config(torch, lib, p4, tree4, 3, 1, 1, 1)
        c4["workload"] = d4
        c4["autotune"] = tune4
        configs["batch_64_molecules"] = c4
        del p4

    out = {
        "metric": METRIC,
        "value": head["dense_interactions_per_s"],
        "unit": "interactions/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 operator, f64 krylov/refinement",
        "data": "synthetic",
        "config": {"workload": desc, "panels": int(n_panels),
                   "gauss_points": int(n_panels * 4), "charges": int(n_charges),
                   "K": 4, "theta": tree["theta"], "P": tree["P"], "tol": 1e-5,
                   "precision": "fp32 bulk, fp64 refinement"},
    }
    out.update({k: v for k, v in head.items() if k not in ("ms_per_step", "rooflines")})
    out["autotune"] = tune
    out["roofline"] = roofline
    out["kernel_rooflines"] = rl
    out["configs"] = configs
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(a.cpu_seconds)
    print(json.dumps(out))
    return 0


if __name__ == "__main__":
    sys.exit(main())
