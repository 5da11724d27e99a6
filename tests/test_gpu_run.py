"""The run command (python -m paper_2312_02968_amd.run) on the two-body workload
(Sect. 4.1): its FP64 diagnostics after a half kick and four steps against the
oracle's half kick and steps, with a zero start and with the warm start."""
import json
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import pm as orc  # noqa: E402
import workloads as W  # noqa: E402
from tests.gpu_util import oparams  # noqa: E402


def oracle_run(warm):
    """The run command's sequence on the oracle: a zero-start half kick with
    the workload's K, then four steps; with the warm start (K = warm) every
    solve after the first starts from H0 = F_prev - g_N, F_prev the last F of
    the previous solve."""
    w = W.two_body()
    p = oparams(w["params"])
    q = oparams(dict(w["params"], iters=warm)) if warm else p
    dt = float(w["dt"])
    pos = w["pos"].astype(np.float64)
    vel = w["vel"].astype(np.float64)
    m = w["mass"].astype(np.float64)
    phi, _ = orc.aqual_solve(p, orc.deposit(p, pos, m))
    pos, vel = orc.interp_push(p, phi, pos, vel, -0.5 * dt, 0.0)
    F_prev = None
    for _ in range(4):
        rho = orc.deposit(q, pos, m)
        H0 = None
        if warm and F_prev is not None:
            H0 = F_prev - orc.newton_potential(q, rho)[1]
        phi, info = orc.aqual_solve(q, rho, H0=H0, keep_fields=True)
        F_prev = info.gN + info.H
        pos, vel = orc.interp_push(q, phi, pos, vel, dt, dt)
    com = (m[:, None] * pos).sum(0) / m.sum()
    return dict(Ekin=0.5 * float((m[:, None] * vel * vel).sum()), mass=float(m.sum()),
                r_mean=float(np.linalg.norm(pos - com, axis=1).mean()))


@pytest.mark.parametrize("warm", [0, 2], ids=["zero_start", "warm2"])
def test_run_two_body(capsys, warm):
    print("run command, two-body, warm", warm, flush=True)
    sys.stdout.flush()
    from paper_2312_02968_amd import run
    argv = ["--workload", "two_body", "--steps", "4", "--every", "2"]
    if warm:
        argv += ["--warm", str(warm)]
    ref = oracle_run(warm)
    capsys.readouterr()
    run.main(argv)
    recs = [json.loads(line) for line in capsys.readouterr().out.splitlines() if line.startswith("{")]
    assert [r["step"] for r in recs] == [0, 2, 4]
    for r in recs:
        assert r["mass"] == ref["mass"]
        assert r["out_of_region"] == 0
        assert r["P_rel"] < 0.05
    assert recs[0]["ms_per_step"] is None and recs[-1]["ms_per_step"] > 0
    assert abs(recs[-1]["Ekin"] - ref["Ekin"]) <= 1e-3 * ref["Ekin"]
    assert abs(recs[-1]["r_mean"] - ref["r_mean"]) <= 1e-4 * ref["r_mean"]
