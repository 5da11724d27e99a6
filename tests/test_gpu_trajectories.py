"""Multi-step runs of the HIP path against FP64 oracle trajectories stored in
tests/golden/trajectories.json (written by tests/golden/make_trajectories.py,
which calls only the oracle): the two-body workload over 200 steps
(Sect. 4.1) and the first 20 steps of the ring workload (Sect. 4.2).

Every step is the same deposit -> solve -> kick -> drift on both sides, from
the same FP32 initial state; FP32 positions drift from the FP64 ones by
rounding (about 1e-5 cell per step at |x| ~ 20).  Trajectories are a
reported result: they are held loosely, to 1e-3 cell and 3e-4 of the
largest speed (measured: 1.7e-6 cell and 2e-7 for the two-body run,
7.4e-6 cell and 5.3e-5 for the ring), and the measured differences are
printed.
"""
import json
import os
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import workloads as W  # noqa: E402
from tests.gpu_util import dev, host  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "trajectories.json")


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_2312_02968_amd import mondpm
    mondpm.lib()
    return mondpm


@pytest.fixture(scope="module")
def golden():
    with open(GOLDEN) as f:
        return json.load(f)


@pytest.mark.parametrize("name,make", [("two_body", W.two_body), ("ring", lambda: W.ring(seed=0))])
def test_trajectory_follows_oracle(M, golden, name, make):
    g = golden[name]
    w = make()
    n = len(w["mass"])
    idx = np.asarray(g["index"])
    ctx = M.pm_create(w["params"], n)
    pos, vel, mass = dev(w["pos"]), dev(w["vel"]), dev(w["mass"])
    scale_v = np.abs(np.asarray(g["vel"][-1])).max()
    worst_x = worst_v = 0.0
    for c in range(1, len(g["pos"])):
        for _ in range(g["every"]):
            M.pm_step(ctx, pos, vel, mass, g["dt"])
        px = host(pos).reshape(-1, 3)[idx]
        pv = host(vel).reshape(-1, 3)[idx]
        dx = np.abs(px - np.asarray(g["pos"][c])).max()
        dv = np.abs(pv - np.asarray(g["vel"][c])).max() / scale_v
        worst_x, worst_v = max(worst_x, dx), max(worst_v, dv)
    _log(f"{name}: {g['steps']} steps, max |dx| {worst_x:.2e} cell, max |dv| / |v| {worst_v:.2e}")
    assert worst_x < 1e-3
    assert worst_v < 3e-4
    ctx.close()
