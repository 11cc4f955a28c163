"""Writes tests/golden/c4_energies.json: the dense FP64 oracle's solvation
energy (LU solve of the assembled system, Eqs. matrix and solv) of every
molecule of the 64-molecule uneven batch (seeds 4000 + i) that has at most
5,120 panels -- 30 molecules of 1,280 to 5,120 panels.

Only the oracle and the seeded input generators are used.

    python tests/golden/make_c4_energies.py
"""

import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import synth  # noqa: E402
from oracle import Oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c4_energies.json")
MAX_PANELS = 5120


def main():
    t0 = time.time()
    mols = synth.config4_batch(n_mol=64)
    out = {"what": "dense FP64 oracle energies, 64-molecule batch (config4_batch), "
                   f"molecules with <= {MAX_PANELS} panels",
           "max_panels": MAX_PANELS, "molecules": []}
    for i, m in enumerate(mols):
        if m.n_panels > MAX_PANELS:
            continue
        o = Oracle(m)
        e = o.solve(use_lu=True).energy
        out["molecules"].append({"index": i, "panels": m.n_panels, "charges": m.n_charges,
                                 "energy_kJmol": e})
        print(f"molecule {i}: {m.n_panels} panels, energy {e:.10f} "
              f"({time.time() - t0:.0f} s)", flush=True)
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(f"wrote {OUT} in {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
