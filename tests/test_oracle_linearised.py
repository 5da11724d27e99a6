"""Pins of the oracle of the linearised incremental update (Sect. 5, item (v)).

- The two linearisations equal central differences of the full algebraic maps
  (Eqs. inverse and interpolation) for all three interpolation functions.
- One iteration on increments is the exact derivative of the one-iteration
  solve started from the previous H.  More iterations match the derivative
  of the full warm solve up to the previous state's distance from a fixed
  point.
- The increment solve is linear in the density increment; with mu = 1 it
  reproduces the Newton solve of the new density exactly.
- Mass scaling of a sphere follows (nu + y nu') g_N.
- FP16 storage of the increments changes them by about FP16's unit roundoff
  and changes the smoothed force of a sphere step far below the 1e-5
  target.
"""
import math

import numpy as np
import pytest

from oracle import linearised as lin
from oracle import pm
import workloads as W

MUS = [pm.MU_STANDARD, pm.MU_DEEP, pm.MU_NEWTON]


def _f64(w):
    return (pm.Params.from_dict(w["params"]), w["pos"].astype(np.float64),
            w["vel"].astype(np.float64), w["mass"].astype(np.float64))


def _q(p, **kw):
    return pm.Params(**{**p.__dict__, **kw})


@pytest.fixture(scope="module", params=[pm.MU_STANDARD, pm.MU_DEEP], ids=["standard", "deep"])
def cloud(request):
    p, pos, vel, m = _f64(W.random_cloud(3, 16, 300, mu=request.param))
    rho = pm.deposit(p, pos, m)
    drho = pm.deposit(p, pos + vel, m) - rho
    return p, rho, drho, lin.base_state(p, rho, max_iters=8)


@pytest.mark.parametrize("mu", MUS, ids=["standard", "deep", "newton"])
def test_linearisations_are_central_differences_of_the_maps(mu):
    rng = np.random.default_rng(11)
    p = pm.Params(n=8, n_pad=8, box=8.0, a0=0.7, mu=mu)
    A = rng.standard_normal((3, 6, 6, 6)) * np.exp(rng.uniform(-3, 3, (1, 6, 6, 6)))
    Am = np.sqrt((A * A).sum(axis=0))
    dA = rng.standard_normal(A.shape) * Am        # a step of the size of each cell's field
    h = 1e-5
    for full, linear in ((pm.apply_nu, lin.linearised_nu), (pm.apply_mu, lin.linearised_mu)):
        fd = (full(p, A + h * dA) - full(p, A - h * dA)) / (2.0 * h)
        got = linear(p, A, dA)
        size = np.sqrt((fd * fd).sum(axis=0))
        assert np.all(np.sqrt(((got - fd) ** 2).sum(axis=0)) <= 1e-7 * size)
        # the slope term matters: without it the MOND maps are not matched
        if mu != pm.MU_NEWTON:
            x = Am / p.a0
            f = lin.nu_value(p, x) if linear is lin.linearised_nu else lin.mu_value(p, x)
            assert np.median(np.sqrt(((f * dA - fd) ** 2).sum(axis=0)) / size) > 1e-2


@pytest.mark.parametrize("mu", MUS[:2], ids=["standard", "deep"])
def test_slopes_in_closed_form(mu):
    # nu(y) y = x solves mu(x) x = y; differentiate the identity: the slope of
    # nu y is 1 / (mu + x mu'), a check that uses neither slope formula
    p = pm.Params(n=8, n_pad=8, box=8.0, a0=1.0, mu=mu)
    y = np.logspace(-4, 4, 41)
    x = lin.nu_value(p, y) * y
    assert np.allclose(lin.mu_value(p, x) * x, y, rtol=1e-12)
    slope = lin.nu_value(p, y) + y * lin.nu_slope(p, y)
    mu_term = lin.mu_value(p, x) + x * lin.mu_slope(p, x)
    assert np.allclose(slope * mu_term, 1.0, rtol=1e-10)


def test_zero_increment_gives_zero(cloud):
    p, rho, _, b = cloud
    d, res = lin.incremental_solve(p, b, np.zeros_like(rho), 3)
    assert not d.any() and res == [0.0, 0.0]


def test_one_iteration_is_the_derivative_of_the_warm_solve(cloud):
    p, rho, drho, b = cloud
    q = _q(p, iters=1, tol=0.0)
    eps = 1e-3
    fd = (pm.aqual_solve(q, rho + eps * drho, H0=b["H"])[0]
          - pm.aqual_solve(q, rho - eps * drho, H0=b["H"])[0]) / (2 * eps)
    d, _ = lin.incremental_solve(p, b, drho, 1)
    assert np.linalg.norm(d - fd) <= 1e-8 * np.linalg.norm(fd)


@pytest.mark.parametrize("K", [2, 3])
def test_more_iterations_follow_the_warm_solve(cloud, K):
    # the linearisation is about the previous F and g_M for every iteration,
    # the full solve's derivative about its own iterates: they differ by the
    # previous state's distance from a fixed point (r ~ 1e-3 here, measured
    # 2-3e-3); an error in the H update moves the result by 0.2-0.4
    p, rho, drho, b = cloud
    assert b["info"].residuals[-1] < 5e-3
    q = _q(p, iters=K, tol=0.0)
    eps = 1e-3
    fd = (pm.aqual_solve(q, rho + eps * drho, H0=b["H"])[0]
          - pm.aqual_solve(q, rho - eps * drho, H0=b["H"])[0]) / (2 * eps)
    d, _ = lin.incremental_solve(p, b, drho, K)
    assert np.linalg.norm(d - fd) <= 1e-2 * np.linalg.norm(fd)


def test_increment_solve_is_linear(cloud):
    p, rho, drho, b = cloud
    rng = np.random.default_rng(5)
    other = pm.deposit(p, rng.uniform(-3, 3, (40, 3)), rng.uniform(0.5, 1.5, 40))
    a, c = 0.37, -1.9
    d1, _ = lin.incremental_solve(p, b, drho, 3)
    d2, _ = lin.incremental_solve(p, b, other, 3)
    d12, _ = lin.incremental_solve(p, b, a * drho + c * other, 3)
    assert np.linalg.norm(d12 - (a * d1 + c * d2)) <= 1e-12 * np.linalg.norm(d12)


def test_newton_increments_are_exact():
    p, pos, vel, m = _f64(W.random_cloud(4, 16, 200, mu=pm.MU_NEWTON))
    rho0 = pm.deposit(p, pos, m)
    rho1 = pm.deposit(p, pos + 3.0 * vel, m)
    b = lin.base_state(p, rho0, max_iters=2)
    d, _ = lin.incremental_solve(p, b, rho1 - rho0, 2)
    phi1, _ = pm.aqual_solve(_q(p, iters=1), rho1)
    assert np.linalg.norm(b["phi"] + d - phi1) <= 1e-12 * np.linalg.norm(phi1)


@pytest.mark.parametrize("mu", MUS[:2], ids=["standard", "deep"])
def test_mass_scaling_of_a_sphere(mu):
    # a spherical mass has g_M = nu(g_N/a0) g_N; scaling the mass by (1 + e)
    # changes it by e (nu + y nu') g_N, with y = g_N/a0: compare the radial
    # field of the increment outside the sphere with that, on the grid's axes
    n = 16
    p = pm.Params(n=n, n_pad=2 * n, box=float(n), a0=0.05, mu=mu, sigma=1.0)
    rho = pm.deposit(p, np.zeros((1, 3)), np.ones(1))
    b = lin.base_state(p, rho, max_iters=6)
    d, _ = lin.incremental_solve(p, b, rho, 3)
    gd = -pm.fd_gradient(p, d)
    gN = b["gN"]
    c = p.n_pad // 2
    for r in (4, 5, 6):                               # cells from the centre, on +x
        gn = -gN[0, c, c, c + r]
        y = gn / p.a0
        want = (lin.nu_value(p, np.array(y)) + y * lin.nu_slope(p, np.array(y))) * gn
        assert abs(-gd[0, c, c, c + r] - want) <= 3e-2 * want
    # the slope term halves the deep-MOND response: a dropped term fails above
    if mu == pm.MU_DEEP:
        assert abs(float(lin.nu_slope(p, np.array(2.0))) * 2.0 / float(lin.nu_value(p, np.array(2.0))) + 0.5) < 1e-12


def test_to_half_rounding():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((3, 8, 8, 8)) * 3e-7
    h = lin.to_half(a)
    scale = 2.0 ** math.ceil(math.log2(np.abs(a).max()))
    normal = np.abs(a) >= scale * 2.0 ** -14
    assert np.all(np.abs(h - a)[normal] <= 2.0 ** -11 * np.abs(a)[normal])
    assert np.all(np.abs(h - a)[~normal] <= scale * 2.0 ** -25)    # half the subnormal spacing
    assert not np.array_equal(h, a)
    assert np.array_equal(lin.to_half(np.array([0.25, -0.5, 1.0])), np.array([0.25, -0.5, 1.0]))
    assert not lin.to_half(np.zeros(4)).any()


def test_half_storage_of_increments(cloud):
    p, rho, drho, b = cloud
    d, _ = lin.incremental_solve(p, b, drho, 2)
    dh, _ = lin.incremental_solve(p, b, drho, 2, store=lin.to_half)
    rel = np.linalg.norm(dh - d) / np.linalg.norm(d)
    assert 1e-6 < rel < 2.0 ** -9


def test_half_storage_on_a_sphere_step():
    # one leapfrog drift of the isothermal sphere (2^12 particles, 32^3 grid):
    # FP16 increments move the smoothed force by < 1e-6 of itself
    p, pos, vel, m = _f64(W.isothermal_sphere(seed=1, N=4096, n=32, b=3.0, r_max=11.0))
    dt = float(W.isothermal_sphere(seed=1, N=16, n=32, b=3.0, r_max=11.0)["dt"])
    rho0 = pm.deposit(p, pos, m)
    pos1 = pos + dt * vel
    drho = pm.deposit(p, pos1, m) - rho0
    b = lin.base_state(p, rho0, max_iters=6)
    d, _ = lin.incremental_solve(p, b, drho, 2)
    dh, _ = lin.incremental_solve(p, b, drho, 2, store=lin.to_half)
    g = pm.smooth_accel(p, b["phi"] + d, pos1)
    gh = pm.smooth_accel(p, b["phi"] + dh, pos1)
    assert np.linalg.norm(gh - g) < 1e-6 * np.linalg.norm(g)


def test_accumulated_newton_increments_are_exact():
    # three steps of increments, each about the base advanced by the last:
    # with mu = 1 the accumulated fields equal the direct solve of the last
    # density (g_N and phi) and F stays g_N + H
    p, pos, vel, m = _f64(W.random_cloud(6, 16, 200, mu=pm.MU_NEWTON))
    rho = pm.deposit(p, pos, m)
    b = lin.base_state(p, rho, max_iters=2)
    for k in range(1, 4):
        rho1 = pm.deposit(p, pos + k * vel, m)
        d, _, inc = lin.incremental_solve(p, b, rho1 - rho, 2, keep_fields=True)
        b = lin.advance_base(b, d, inc)
        rho = rho1
    phi1, _ = pm.aqual_solve(_q(p, iters=1), rho)
    _, gN1 = pm.newton_potential(p, rho)
    assert np.linalg.norm(b["phi"] - phi1) <= 1e-12 * np.linalg.norm(phi1)
    assert np.linalg.norm(b["gN"] - gN1) <= 1e-12 * np.linalg.norm(gN1)
    assert np.linalg.norm(b["F"] - (b["gN"] + b["H"])) <= 1e-14 * np.linalg.norm(b["F"])


def test_accumulated_half_increments_drift_slowly():
    # five drifts of the isothermal sphere (2^12 particles, 32^3 grid), the
    # base advanced by the increments each step: FP16 storage moves the
    # smoothed force from the FP64 chain's by < 1e-6 (measured 7e-8 per step
    # at first, 2.2e-7 after 20 steps)
    w = W.isothermal_sphere(seed=1, N=4096, n=32, b=3.0, r_max=11.0)
    p, pos, vel, m = _f64(w)
    dt = float(w["dt"])
    rho = pm.deposit(p, pos, m)
    b64 = lin.base_state(p, rho, max_iters=6)
    b16 = dict(b64)
    for _ in range(5):
        pos = pos + dt * vel
        rho1 = pm.deposit(p, pos, m)
        d64, _, i64 = lin.incremental_solve(p, b64, rho1 - rho, 2, keep_fields=True)
        d16, _, i16 = lin.incremental_solve(p, b16, rho1 - rho, 2, store=lin.to_half, keep_fields=True)
        b64 = lin.advance_base(b64, d64, i64)
        b16 = lin.advance_base(b16, d16, i16)
        rho = rho1
    g64 = pm.smooth_accel(p, b64["phi"], pos)
    g16 = pm.smooth_accel(p, b16["phi"], pos)
    assert 0.0 < np.linalg.norm(g16 - g64) < 1e-6 * np.linalg.norm(g64)


def test_base_gM_is_the_field_of_the_potential(cloud):
    # the last projection gives phi_hat = i At kt . g and g_M = -i kt phi_hat,
    # so the base g_M is the spectral field of the base potential: the GPU
    # forms the base of the second linearisation that way from phi
    p, rho, _, b = cloud
    _, kt = pm.wavevectors(p)
    ph = pm.fft3(b["phi"])
    g = np.stack([pm.ifft3_real(-1j * k * ph) for k in (kt[None, None, :], kt[None, :, None], kt[:, None, None])])
    assert np.linalg.norm(g - b["gM"]) <= 1e-12 * np.linalg.norm(b["gM"])
    # it is not the central-difference field (the projections use the true k)
    assert np.linalg.norm(-pm.fd_gradient(p, b["phi"]) - b["gM"]) > 1e-3 * np.linalg.norm(b["gM"])
