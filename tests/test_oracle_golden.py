"""The oracle reproduces its stored fixed-schedule trajectory (CPU only)."""
import json
import os

import numpy as np

import fde_synth
from oracle import scf

HERE = os.path.dirname(os.path.abspath(__file__))


def test_c1_trajectory_regression():
    with open(os.path.join(HERE, "golden", "c1_trajectory.json")) as f:
        ref = json.load(f)
    s = fde_synth.config1()
    recs, _, st = scf.run(s)
    assert st.spheres[0].npw == ref["npw"] == 895
    for c, r in enumerate(recs):
        for I in range(2):
            assert np.max(np.abs(r.eps[I].ravel() - np.array(ref["eps"][c][I]))) < 1e-11
            assert abs(r.rho_out[I].sum() * st.cell.dV - 4.0) < 1e-12
