"""Writes tests/golden/trajectories.json: FP64 oracle trajectories of the
two-body workload (200 steps, Sect. 4.1) and of the ring workload (the first
20 steps, Sect. 4.2), from the seeded FP32 initial states of `workloads`.

Only the oracle computes here.  The GPU tests run the same steps through the
C ABI and compare the checkpointed positions and velocities.

    python tests/golden/make_trajectories.py     # about 20 minutes on 8 cores
"""
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from oracle import pm as orc  # noqa: E402
import workloads as W  # noqa: E402

RING_SAMPLE = list(range(0, 4097, 64))      # the central mass and 64 ring particles


def run(w, steps, every, sample=None):
    p = orc.Params.from_dict(w["params"])
    pos = w["pos"].astype(np.float64)
    vel = w["vel"].astype(np.float64)
    mass = w["mass"].astype(np.float64)
    idx = np.arange(len(mass)) if sample is None else np.asarray(sample)
    out = {"steps": steps, "every": every, "dt": float(w["dt"]), "index": idx.tolist(),
           "pos": [pos[idx].tolist()], "vel": [vel[idx].tolist()], "residual_last": []}
    t0 = time.time()
    for k in range(1, steps + 1):
        pos, vel, info = orc.pm_step(p, pos, vel, mass, float(w["dt"]))
        if k % every == 0:
            out["pos"].append(pos[idx].tolist())
            out["vel"].append(vel[idx].tolist())
            out["residual_last"].append(info.residuals[-1] if info.residuals else 0.0)
            print(f"{w['workload']}: step {k} ({time.time() - t0:.0f} s)", flush=True)
    return out


def main():
    res = {"two_body": run(W.two_body(), 200, 10),
           "ring": run(W.ring(seed=0), 20, 5, RING_SAMPLE)}
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "trajectories.json")
    with open(path, "w") as f:
        json.dump(res, f)
    print("wrote", path)


if __name__ == "__main__":
    main()
