"""Writes tests/golden/mlp_params.npy: the learned preconditioner's parameters.

Trained offline with the FP64 oracle only (oracle.mlp: features, Jacobi-Davidson
corrections solved against the dense H of small cells, the hand-written backward
pass and Adam), on the rows of tests/mlp_harvest.py (12 seeded 8 x 8 x 9 bohr
cells). The GPU library trains the same network with its own kernels in
tests/test_gpu_mlp_gain.py; this file only fixes one trained parameter set for
the benchmark's band-solver comparison, so the benchmark calls no oracle code.

    python tests/golden/make_mlp_params.py
"""
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))
sys.path.insert(0, os.path.dirname(HERE))

import fde_synth  # noqa: E402
import mlp_harvest as mh  # noqa: E402
from oracle import mlp  # noqa: E402


def main(steps=300, lr=3e-3):
    S = mh.harvest(range(12)).astype(np.float64)
    th = fde_synth.mlp_init(0)
    m = np.zeros_like(th)
    v = np.zeros_like(th)
    l0 = mlp.loss(th, S)
    for t in range(1, steps + 1):
        L, g = mlp.loss_grad(th, S)
        th, m, v = mlp.adam(th, g, m, v, t, lr)
        if t % 50 == 0:
            print(f"step {t}: loss {L:.5f}", flush=True)
    l1 = mlp.loss(th, S)
    np.save(os.path.join(HERE, "mlp_params.npy"), th.astype(np.float32))
    with open(os.path.join(HERE, "mlp_params.json"), "w") as f:
        json.dump({"rows": int(S.shape[0]), "steps": steps, "lr": lr, "loss_tpa": l0, "loss_trained": l1}, f,
                  indent=1)
    print(f"loss {l0:.5f} (TPA) -> {l1:.5f}")


if __name__ == "__main__":
    main()
