"""Writes tests/golden/c5_gradient.json: the dense FP64 oracle's energy and
exact discrete gradients (dE/dq, dE/dkappa, dE/deps per region) of the
reduced three-region system -- protein and Stern layer at icosahedral
nu = 16 (5,120 panels each), two cavities at octahedral nu = 8 (512 each),
4,000 charges, 22,528 unknowns.

Only the oracle and the seeded input generators are used (the adjoint
formulas of the oracle follow Eqs. matrix, reac_integral and solv).  The
dense matrices take about 20 GB of host memory; run time is several minutes.

    python tests/golden/make_c5_gradient.py
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import Oracle  # noqa: E402
from oracle.adjoint import gradients  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c5_gradient.json")


def main():
    t0 = time.time()
    prob = synth.config5_small()
    o = Oracle(prob)
    print(f"{o.n} unknowns, {len(o.q)} charges", flush=True)
    g = gradients(o)
    out = {
        "what": "dense FP64 oracle, reduced three-region system (config5_small)",
        "K": o.par.k, "K_fine": o.par.k_fine, "N_k": o.par.nk, "thres": o.par.thres,
        "n_unknowns": int(o.n), "n_charges": int(len(o.q)),
        "regions": [r.name for r in prob.regions],
        "energy_kJmol": g["energy"],
        "dE_dq": [float(v) for v in g["dE_dq"]],
        "dE_dkappa": [float(v) for v in g["dE_dkappa"]],
        "dE_deps": [float(v) for v in g["dE_deps"]],
        "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(out, f)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s: energy {g['energy']:.10f}", flush=True)


if __name__ == "__main__":
    main()
