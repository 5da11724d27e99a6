"""Pins of the oracle's diagnostics (the constants of motion of Sect. 4.1), of
the particle-smoothed potential, and of two statements the paper makes about
the method as a whole: the angular-momentum error of the two-body orbit
(Sect. 4.1) and "four iterations give 1 %" (Abstract, Sect. 6)."""
import math

import numpy as np

from oracle import pm
from tests import analytic as A


def test_diagnostics_hand_computed():
    # Three particles on the axes, each moving along another axis.  By hand:
    #   P = 1 (0,1,0) + 2 (0,0,1) + 3 (1,0,0) = (3, 1, 2)
    #   r1 x v1 = (1,0,0) x (0,1,0) = (0,0,1)       -> 1 (0,0,1)
    #   r2 x v2 = (0,2,0) x (0,0,1) = (2,0,0)       -> 2 (2,0,0)
    #   r3 x v3 = (0,0,3) x (1,0,0) = (0,3,0)       -> 3 (0,3,0)
    #   L = (4, 9, 1);  E_kin = (1 + 2 + 3) / 2 = 3;  mass = 6.
    pos = np.array([[1.0, 0.0, 0.0], [0.0, 2.0, 0.0], [0.0, 0.0, 3.0]])
    vel = np.array([[0.0, 1.0, 0.0], [0.0, 0.0, 1.0], [1.0, 0.0, 0.0]])
    mass = np.array([1.0, 2.0, 3.0])
    p = pm.Params(n=8, n_pad=16, box=8.0)
    d = pm.diagnostics(p, pos, vel, mass)
    assert np.array_equal(d["P"], [3.0, 1.0, 2.0])
    assert np.array_equal(d["L"], [4.0, 9.0, 1.0])
    assert d["Ekin"] == 3.0
    assert d["mass"] == 6.0
    assert "Epot_sum" not in d


def _grid_coords(p):
    N = p.n_pad
    ax = (np.arange(N) - N // 2) * p.s
    return np.meshgrid(ax, ax, ax, indexing="ij")      # z, y, x


def test_potential_at_particles_constant_and_linear():
    # The normalised weights sum to one, so a constant potential is returned
    # exactly; for a particle on a grid point the ball is symmetric about it,
    # so a linear potential a.x returns a.x_i exactly.
    p = pm.Params(n=16, n_pad=32, box=24.0, sigma=1.5)    # s = 1.5
    z, y, x = _grid_coords(p)
    rng = np.random.default_rng(3)
    off = rng.uniform(-6.0, 6.0, (10, 3))
    assert np.max(np.abs(pm.potential_at_particles(p, np.full(x.shape, -2.5), off) + 2.5)) < 1e-14
    on = rng.integers(-4, 5, (10, 3)) * p.s
    a = np.array([0.4, -1.1, 2.3])
    phi = a[0] * x + a[1] * y + a[2] * z
    assert np.max(np.abs(pm.potential_at_particles(p, phi, on) - on @ a)) < 1e-12


def test_smoothed_potential_is_the_adjoint_of_the_deposit():
    # Deposit and smoothing share the weights: s^3 rho_c = sum_i m_i w_ic, so
    # sum_i m_i phi~(r_i) = s^3 sum_c rho_c phi_c for any phi (also for balls
    # that wrap around the periodic box).
    p = pm.Params(n=8, n_pad=16, box=12.0, sigma=1.0)
    rng = np.random.default_rng(11)
    N = p.n_pad
    phi = rng.standard_normal((N, N, N))
    pos = rng.uniform(-9.0, 9.0, (40, 3))                # some balls wrap
    mass = rng.uniform(0.5, 2.0, 40)
    lhs = float((mass * pm.potential_at_particles(p, phi, pos)).sum())
    rhs = float((pm.deposit(p, pos, mass) * phi).sum()) * p.s ** 3
    assert abs(lhs - rhs) < 1e-11 * (abs(rhs) + 1.0)
    vel = rng.standard_normal((40, 3))
    assert abs(pm.diagnostics(p, pos, vel, mass, phi)["Epot_sum"] - lhs) < 1e-12 * (abs(lhs) + 1.0)


def test_two_body_angular_momentum_within_the_papers_error(golden):
    # Sect. 4.1: the total angular momentum of the deep-MOND two-body orbit
    # (m1/m2 = 3/2) is conserved to 4 % on the coarsest grid the paper shows,
    # the error coming from the cubic mesh.  Here: an eccentric orbit (80 % of
    # the circular speed at 8 cells, from the closed-form force of
    # Eq. twobodyforce) on a 32^3 grid, sigma = 1, K = 4, one period in 60
    # steps.
    G, a0, m1, m2 = 1.0, 1e3, 1.5, 1.0
    M, r0 = m1 + m2, 8.0
    F = A.two_body_force(m1, m2, r0, G, a0)
    vrel = 0.8 * math.sqrt(F * r0 / (m1 * m2 / M))
    pos = np.array([[-r0 * m2 / M, 0.0, 0.0], [r0 * m1 / M, 0.0, 0.0]])
    vel = np.array([[0.0, -vrel * m2 / M, 0.0], [0.0, vrel * m1 / M, 0.0]])
    mass = np.array([m1, m2])
    p = pm.Params(n=32, n_pad=64, box=32.0, G=G, a0=a0, mu=pm.MU_DEEP, sigma=1.0, iters=4)
    steps = 60
    dt = 2.0 * math.pi * r0 / vrel / steps
    phi, _ = pm.aqual_solve(p, pm.deposit(p, pos, mass))
    pos, vel = pm.interp_push(p, phi, pos, vel, -0.5 * dt, 0.0)
    L0 = pm.diagnostics(p, pos, vel, mass)["L"]
    worst = 0.0
    for _ in range(steps):
        pos, vel, _ = pm.pm_step(p, pos, vel, mass, dt)
        L = pm.diagnostics(p, pos, vel, mass)["L"]
        worst = max(worst, float(np.linalg.norm(L - L0) / np.linalg.norm(L0)))
    bound = golden["angular_momentum_error"]["percent"][0] / 100.0
    assert 0.0 < worst < bound, worst


def _sphere_and_two_body():
    import workloads as W
    cases = []
    w = W.isothermal_sphere(seed=0, N=1 << 12, n=32, b=4.0, r_max=14.0)
    cases.append((pm.Params.from_dict(w["params"]), w["pos"].astype(np.float64), w["mass"].astype(np.float64)))
    w = W.two_body()
    p = pm.Params.from_dict({**w["params"], "n": 32, "n_pad": 64, "box": 32.0})
    cases.append((p, w["pos"].astype(np.float64), w["mass"].astype(np.float64)))
    return cases


def test_four_iterations_give_one_percent(golden):
    # Abstract and Sect. 6: four iterations give a force within 1 % of the
    # converged one.  The smoothed particle forces after K = 4 agree with
    # K = 20 to 1 % on a standard-mu sphere and on the deep-MOND two-body
    # system; one iteration does not reach 1 % on the two-body system.
    K = golden["iterations_for_one_percent"]["value"]
    for i, (p, pos, mass) in enumerate(_sphere_and_two_body()):
        rho = pm.deposit(p, pos, mass)
        acc = {}
        for k in (1, K, 20):
            q = pm.Params(**{**p.__dict__, "iters": k})
            phi, _ = pm.aqual_solve(q, rho)
            acc[k] = pm.smooth_accel(q, phi, pos)
        err = {k: float(np.linalg.norm(acc[k] - acc[20]) / np.linalg.norm(acc[20])) for k in (1, K)}
        assert err[K] < 1e-2, (i, err)
        if i == 1:
            assert err[1] > 1e-2, err


def test_late_iterates_alternate_on_the_grid_scale():
    # Reading of the convergence statement of Sect. 2.1: on this
    # discretisation the undamped iteration does not run to machine precision.
    # After four to six iterations successive H differ by a fixed amount while
    # every other iterate nearly repeats (a period-two alternation), and what
    # alternates lies at high wavenumbers, largest at the sphere's centre where
    # F vanishes and nu(|F|/a0) is unbounded.  r_k = ||H_k - H_{k-1}|| / ||g_N||
    # therefore stalls near 6e-4 here and never reaches 1e-5.
    p, pos, mass = _sphere_and_two_body()[0]
    _, gN = pm.newton_potential(p, pm.deposit(p, pos, mass))
    H = np.zeros_like(gN)
    Hs = [H]
    for _ in range(16):
        gM = pm.apply_nu(p, gN + H)
        gh, _ = pm.project_curl_free(p, np.stack([pm.fft3(c) for c in gM]))
        Fp = pm.apply_mu(p, np.stack([pm.ifft3_real(c) for c in gh]))
        Hh = pm.project_div_free(p, np.stack([pm.fft3(c) for c in Fp - gN]))
        H = np.stack([pm.ifft3_real(c) for c in Hh])
        Hs.append(H)
    nG = math.sqrt(float((gN * gN).sum()))
    r1 = [math.sqrt(float(((Hs[k] - Hs[k - 1]) ** 2).sum())) / nG for k in range(1, 17)]
    r2 = [math.sqrt(float(((Hs[k] - Hs[k - 2]) ** 2).sum())) / nG for k in range(2, 17)]
    assert r1[1] < 0.2 * r1[0] and r1[2] < 0.3 * r1[1]          # the early drop
    assert min(r1) > 1e-4                                       # no convergence below 1e-4
    assert max(r1[8:]) < 2.0 * min(r1)                          # a stall, not a divergence
    assert r2[-1] < 0.05 * r1[-1]                               # every other iterate repeats
    d = Hs[-1] - Hs[-2]
    N = p.n_pad
    P = sum(np.abs(np.fft.fftn(c)) ** 2 for c in d)
    m = np.abs(np.fft.fftfreq(N, 1.0 / N))
    mmax = np.maximum(np.maximum(m[None, None, :], m[:, None, None]), m[None, :, None])
    assert P[mmax >= N // 4].sum() > 0.7 * P.sum()              # upper half of the band
    amp = np.sqrt((d * d).sum(axis=0))
    peak = np.array(np.unravel_index(np.argmax(amp), amp.shape)) - N // 2
    assert np.all(np.abs(peak) <= 1)                            # at the centre
