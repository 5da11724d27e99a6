"""Advance a workload with pm_step and print its FP64 constants of motion.

    python -m paper_2312_02968_amd.run [--workload isothermal] [--steps 100]
                                       [--every 10] [--warm K]

Starts with the half kick that puts the velocities half a step behind the
positions (leapfrog, Sect. 3), then runs the steps.  Every `every` steps it
prints one JSON line with the total momentum P, angular momentum L, kinetic
energy, mass, sum m_i phi_i and the number of particles whose ball leaves the
physical region (pm_diagnostics), and the particles' mean distance from the
centre of mass, its spread (standard deviation) and their mean speed.  The
half kick and the diagnostics solve
with the workload's own iterations from a zero start, in a context of their
own, so that they leave the warm start of the stepping context alone.  The
momentum is reported relative to
sum m |v|: the MOND step does not conserve it exactly (the paper's method is
not variational), so its drift is a measured property of the run.
"""
import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2312_02968_amd import mondpm as M  # noqa: E402
import workloads as W  # noqa: E402

WORKLOADS = {
    "isothermal": lambda: W.isothermal_sphere(seed=0),
    "two_body": W.two_body,
    "ring": lambda: W.ring(seed=0),
    "plummer512": lambda: W.plummer_mixture(seed=0),
}


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", default="isothermal", choices=sorted(WORKLOADS))
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--every", type=int, default=10)
    ap.add_argument("--warm", type=int, default=0, metavar="K",
                    help="warm start (previous step's field) with K iterations")
    a = ap.parse_args(argv)
    w = WORKLOADS[a.workload]()
    p0 = dict(w["params"])
    p = dict(p0)
    if a.warm:
        p.update(iters=a.warm, flags=p.get("flags", 0) | M.PM_F_WARM_START)
    dt = float(w["dt"])
    n = len(w["mass"])
    torch.cuda.init()
    ctx = M.pm_create(p, n)
    dctx = M.pm_create(p0, n)                 # half kick and diagnostics
    pos = torch.from_numpy(w["pos"]).cuda()
    vel = torch.from_numpy(w["vel"]).cuda()
    mass = torch.from_numpy(w["mass"]).cuda()
    # half kick: v(-dt/2) from the force at the initial positions
    N = p["n_pad"]
    rho = torch.zeros(N ** 3, device="cuda")
    phi = torch.zeros_like(rho)
    M.pm_deposit(dctx, pos, mass, rho)
    M.aqual_solve(dctx, rho, phi, want_info=False)
    M.interp_push(dctx, phi, pos, vel, -0.5 * dt, 0.0)

    def report(step, t_ms):
        M.pm_deposit(dctx, pos, mass, rho)
        M.aqual_solve(dctx, rho, phi, want_info=False)
        d = M.pm_diagnostics(dctx, pos, vel, mass, phi)
        v = vel.double().reshape(-1, 3)
        scale = float((mass.double()[:, None] * v.abs()).sum())
        x = pos.double().reshape(-1, 3)
        md = mass.double()
        com = (md[:, None] * x).sum(0) / md.sum()
        r = torch.linalg.vector_norm(x - com, dim=1)
        rec = {"step": step, "P_rel": float(np.linalg.norm(d["P"])) / scale, "L": d["L"],
               "Ekin": d["Ekin"], "mass": d["mass"], "Epot_sum": d["Epot_sum"],
               "out_of_region": d["out_of_region"], "r_mean": float(r.mean()), "r_std": float(r.std()),
               "v_mean": float(torch.linalg.vector_norm(v, dim=1).mean()), "ms_per_step": t_ms}
        print(json.dumps(rec), flush=True)

    report(0, None)
    done = 0
    while done < a.steps:
        k = min(a.every, a.steps - done)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(k):
            M.pm_step(ctx, pos, vel, mass, dt)
        torch.cuda.synchronize()
        t = (time.perf_counter() - t0) * 1e3 / k
        done += k
        report(done, round(t, 3))
    ctx.close()
    dctx.close()


if __name__ == "__main__":
    main()
