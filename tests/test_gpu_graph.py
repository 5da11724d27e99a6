"""One PM step recorded as a HIP graph (pm_step_capture / pm_step_replay) against
eager pm_step calls and the FP64 oracle.

Every replay is checked against an eager step of the same state, with eager
work and host synchronisations between replays.  Eager and replayed steps
differ only in the order of the deposit's atomic additions, so they agree to
FP32 rounding; the first replay is also held to the force tolerance (1e-5
relative) against the oracle's step.
"""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import pm as orc  # noqa: E402
import workloads as W  # noqa: E402
from tests.gpu_util import dev, host, oparams, rel_l2, rel_max  # noqa: E402


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_2312_02968_amd import mondpm
    mondpm.lib()
    return mondpm


def _state(w):
    return dev(w["pos"]), dev(w["vel"]), dev(w["mass"])


def _agree(a_pos, a_vel, b_pos, b_vel, vel0):
    pa, pb = host(a_pos).reshape(-1, 3), host(b_pos).reshape(-1, 3)
    va, vb = host(a_vel).reshape(-1, 3), host(b_vel).reshape(-1, 3)
    assert rel_l2(vb - vel0, va - vel0) < 1e-5
    assert np.max(np.abs(pb - pa)) < 1e-5 * max(1.0, np.abs(pa).max())


CASES = [
    ("iso_small", lambda: W.isothermal_sphere(seed=1, N=4096, n=32, b=3.0, r_max=11.0)),
    ("cloud_deep", lambda: W.random_cloud(32, 32, 400, mu=1, radius_frac=0.2)),
]


@pytest.mark.parametrize("name,make", CASES, ids=[c[0] for c in CASES])
def test_replay_matches_eager_and_oracle(M, name, make):
    _log("graph replay", name)
    w = make()
    p = w["params"]
    n_p = len(w["mass"])
    dt = float(w["dt"])
    s = torch.cuda.Stream()
    ctx = M.pm_create(p, n_p, stream=s)
    pos_e, vel_e, mass_e = _state(w)
    pos_g, vel_g, mass_g = _state(w)
    torch.cuda.synchronize()
    M.pm_step_capture(ctx, pos_g, vel_g, mass_g, dt)
    torch.cuda.synchronize()
    # capturing records the step without running it
    assert np.array_equal(host(pos_g).reshape(-1, 3), w["pos"].astype(np.float64))
    assert np.array_equal(host(vel_g).reshape(-1, 3), w["vel"].astype(np.float64))
    pr, vr, _ = orc.pm_step(oparams(p), w["pos"].astype(np.float64), w["vel"].astype(np.float64),
                            w["mass"].astype(np.float64), dt)
    vel0 = w["vel"].astype(np.float64)
    for r in range(3):
        M.pm_step_replay(ctx, 1)
        M.pm_step(ctx, pos_e, vel_e, mass_e, dt)
        torch.cuda.synchronize()
        if r == 0:
            g_ref = (vr - vel0) / dt
            g = (host(vel_g).reshape(-1, 3) - vel0) / dt
            assert rel_l2(g, g_ref) < 1e-5
            assert rel_max(g, g_ref) < 1e-5
        _agree(pos_e, vel_e, pos_g, vel_g, vel0)
    # several replays in one call
    M.pm_step_replay(ctx, 2)
    for _ in range(2):
        M.pm_step(ctx, pos_e, vel_e, mass_e, dt)
    torch.cuda.synchronize()
    _agree(pos_e, vel_e, pos_g, vel_g, vel0)
    ctx.close()


def test_replay_with_warm_start(M):
    _log("graph replay warm start")
    w = W.isothermal_sphere(seed=2, N=4096, n=32, b=3.0, r_max=11.0)
    p = dict(w["params"], iters=2, flags=M.PM_F_WARM_START)
    n_p = len(w["mass"])
    dt = float(w["dt"])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ce = M.pm_create(p, n_p, stream=s1)
    cg = M.pm_create(p, n_p, stream=s2)
    pos_e, vel_e, mass_e = _state(w)
    pos_g, vel_g, mass_g = _state(w)
    torch.cuda.synchronize()
    with pytest.raises(M.PmError):                   # no previous solve to start from yet
        M.pm_step_capture(cg, pos_g, vel_g, mass_g, dt)
    M.pm_step(ce, pos_e, vel_e, mass_e, dt)
    M.pm_step(cg, pos_g, vel_g, mass_g, dt)
    torch.cuda.synchronize()
    M.pm_step_capture(cg, pos_g, vel_g, mass_g, dt)
    vel0 = w["vel"].astype(np.float64)
    for _ in range(3):
        M.pm_step_replay(cg, 1)
        M.pm_step(ce, pos_e, vel_e, mass_e, dt)
        torch.cuda.synchronize()
        _agree(pos_e, vel_e, pos_g, vel_g, vel0)
    ce.close()
    cg.close()


def test_capture_argument_checks(M):
    w = W.random_cloud(33, 16, 50, mu=0)
    p = w["params"]
    s = torch.cuda.Stream()
    pos, vel, mass = _state(w)
    torch.cuda.synchronize()
    ctx = M.pm_create(p, 50, stream=s)
    with pytest.raises(M.PmError):                   # nothing captured yet
        M.pm_step_replay(ctx, 1)
    M.pm_set_timing(ctx, True)
    with pytest.raises(M.PmError):                   # event timing on
        M.pm_step_capture(ctx, pos, vel, mass, 0.1)
    M.pm_set_timing(ctx, False)
    M.pm_step_capture(ctx, pos, vel, mass, 0.1)
    with pytest.raises(M.PmError):
        M.pm_step_replay(ctx, -1)
    M.pm_step_replay(ctx, 0)
    ctx.close()
    if torch.cuda.current_stream().cuda_stream == 0:
        cnull = M.pm_create(p, 50)
        with pytest.raises(M.PmError):               # the null stream cannot be captured
            M.pm_step_capture(cnull, pos, vel, mass, 0.1)
        cnull.close()
    torch.cuda.synchronize()


def test_replay_keeps_the_external_field_of_capture(M):
    # the sheets' density is a kernel argument of the captured Newton pass:
    # changing the context's field later does not change the replayed step
    _log("graph replay with an external field")
    w = W.isothermal_sphere(seed=3, N=4096, n=32, b=3.0, r_max=11.0)
    p = w["params"]
    n_p = len(w["mass"])
    dt = float(w["dt"])
    g = (0.0, 0.3 * p["a0"], 0.2 * p["a0"])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ce = M.pm_create(p, n_p, stream=s1)
    cg = M.pm_create(p, n_p, stream=s2)
    M.pm_set_external_field(ce, g)
    M.pm_set_external_field(cg, g)
    pos_e, vel_e, mass_e = _state(w)
    pos_g, vel_g, mass_g = _state(w)
    torch.cuda.synchronize()
    M.pm_step_capture(cg, pos_g, vel_g, mass_g, dt)
    M.pm_set_external_field(cg, (0.0, 0.0, 0.0))
    vel0 = w["vel"].astype(np.float64)
    for _ in range(2):
        M.pm_step_replay(cg, 1)
        M.pm_step(ce, pos_e, vel_e, mass_e, dt)
        torch.cuda.synchronize()
        _agree(pos_e, vel_e, pos_g, vel_g, vel0)
    # and the field changed the steps: the same two eager steps without it differ
    pos_z, vel_z, mass_z = _state(w)
    cz = M.pm_create(p, n_p, stream=s1)
    torch.cuda.synchronize()
    for _ in range(2):
        M.pm_step(cz, pos_z, vel_z, mass_z, dt)
    torch.cuda.synchronize()
    v1 = host(vel_z).reshape(-1, 3) - vel0
    ve = host(vel_e).reshape(-1, 3) - vel0
    assert rel_l2(v1, ve) > 1e-2
    ce.close()
    cg.close()
    cz.close()


def test_tolerance_mode_on_the_device(M):
    """The tolerance mode decides on the device: a tol solve equals, bit for
    bit, the fixed-K solve with the K it reports (the gates skip exactly the
    passes after the stop), and a replayed tol step follows eager tol steps."""
    _log("tolerance mode on the device")
    w = W.random_cloud(34, 32, 2000, mu=0)
    p = dict(w["params"], tol=5e-3, iters=12)
    n_p = len(w["mass"])
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    ct = M.pm_create(p, n_p, stream=s1)
    N = ct.N
    pos, vel, mass = _state(w)
    rho = torch.zeros(N ** 3, device="cuda")
    M.pm_deposit(ct, pos, mass, rho)
    phi_t = torch.zeros_like(rho)
    info = M.aqual_solve(ct, rho, phi_t)
    k = info["iterations"]
    _log(f"  stopped after {k} iterations, residuals {info['residuals']}")
    assert 2 <= k < 12 and info["status"] == 0
    assert info["residuals"][-1] <= 5e-3 and all(r > 5e-3 for r in info["residuals"][:-1])
    cf = M.pm_create(dict(p, tol=0.0, iters=k, flags=M.PM_F_RESIDUAL), n_p, stream=s1)
    phi_f = torch.zeros_like(rho)
    info_f = M.aqual_solve(cf, rho, phi_f)
    assert torch.equal(phi_t, phi_f)
    assert info_f["residuals"] == info["residuals"]
    cf.close()
    # a graph of tol steps against eager tol steps
    cg = M.pm_create(p, n_p, stream=s2)
    gpos, gvel, _ = _state(w)
    epos, evel, _ = _state(w)
    vel0 = host(evel).reshape(-1, 3)
    torch.cuda.synchronize()
    M.pm_step_capture(cg, gpos, gvel, mass, float(w["dt"]))
    for step in range(3):
        M.pm_step(ct, epos, evel, mass, float(w["dt"]))
        M.pm_step_replay(cg, 1)
        torch.cuda.synchronize()
        _agree(epos, evel, gpos, gvel, vel0)
    ct.close()
    cg.close()
