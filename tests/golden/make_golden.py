"""Writes tests/golden/c1_trajectory.json from the CPU oracle only.

The paper prints no worked numerical example for any step of the method
(its Table 1 needs pseudopotential files and geometries that are not
available), so the stored values here are the oracle's own fixed-schedule
trajectory on the two-subsystem 24^3 cell: eigenvalues and charges per cycle.
They guard the oracle against unintended changes and give the GPU trajectory
test a stored reference. Run: python tests/golden/make_golden.py
"""
import json
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fde_synth  # noqa: E402
from oracle import scf  # noqa: E402


def main():
    s = fde_synth.config1()
    recs, X, st = scf.run(s)
    out = {
        "system": "two 2-atom subsystems, L=10 bohr cube, 24^3 grid, E_cut=7 Ha, Gamma, LDA + TF*LC94",
        "schedule": {"cycles": s.n_cycles, "davidson": s.n_david, "mix_beta": s.mix_beta},
        "npw": int(st.spheres[0].npw),
        "eps": [[r.eps[I].ravel().tolist() for I in range(len(s.subsystems))] for r in recs],
        "mu": [list(map(float, r.mu)) for r in recs],
        "charge_out": [[float(r.rho_out[I].sum() * st.cell.dV) for I in range(len(s.subsystems))] for r in recs],
    }
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_trajectory.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
