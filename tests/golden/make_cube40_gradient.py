"""Writes cube40_gradient.json: the oracle's reference gradient of the final kinetic
energy of the 64,000-particle cube (40^3 lattice, dx = 1/16, 20 kick-drift-kick steps,
dt = 0.2 dx / c) with respect to the initial velocities, mu and Y0.

Calls only the oracle (reverse-mode AD of its torch transcription, partner sets by
brute force at every evaluation).  Takes a few minutes and ~25 GB of host memory:
    python tests/golden/make_cube40_gradient.py
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import autodiff as AD  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube40_gradient.json")
DIRECTION_SEED = 4040
SAMPLE_SEED = 4041


def main():
    w = W.config(3)
    t0 = time.time()
    g = AD.leapfrog_grad(w, w.steps, w.dt, "ke")
    d = np.random.default_rng(DIRECTION_SEED).normal(size=w.vel.shape)
    idx = W.subsample(w.n, 64, SAMPLE_SEED)
    out = {
        "workload": w.name, "n": w.n, "steps": w.steps, "dt": w.dt, "objective": "ke",
        "direction_seed": DIRECTION_SEED, "sample_seed": SAMPLE_SEED,
        "J": g["J"], "mu": g["mu"], "Y0": g["Y0"],
        "v0_dot_direction": float((g["v0"] * d).sum()),
        "sample_index": idx.tolist(), "v0_sample": g["v0"][:, idx].tolist(),
        "seconds": time.time() - t0,
    }
    with open(OUT, "w") as f:
        json.dump(out, f, indent=1)
    print(OUT, out["seconds"])


if __name__ == "__main__":
    main()
