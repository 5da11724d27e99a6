"""Pins of the oracle's field solve: DFT conventions, Newton solve, the AQUAL
fixed-point iteration (Sect. 2.1 and the flow scheme), the interpolation pair
and the paper's analytic cases."""
import math

import numpy as np
import pytest

from oracle import pm
import workloads as W
from tests import analytic as A


def test_fft_matches_brute_force_dft():
    # Appendix 'Fourier transforms': f_hat(k) = sum_r f(r) exp(-i k.r) (times
    # s^3) and the inverse with 1/L^3; brute force on 8^3.
    rng = np.random.default_rng(0)
    N = 8
    f = rng.standard_normal((N, N, N))
    j = np.arange(N)
    E = np.exp(-2j * np.pi * np.outer(j, j) / N)
    brute = np.einsum("az,by,cx,zyx->abc", E, E, E, f)
    got = pm.fft3(f)
    assert np.max(np.abs(got - brute)) < 1e-12 * np.max(np.abs(brute))
    back = pm.ifft3_real(got)
    assert np.max(np.abs(back - f)) < 1e-13


def test_newton_single_mode_closed_form():
    # rho = cos(k.x) solves grad^2 phi = 4 pi G rho with phi = -4 pi G cos(k.x)/k^2;
    # the central difference of cos gives -sin(k.x) sin(k_d s)/s.
    p = pm.Params(n=8, n_pad=16, box=4.0, G=0.7)          # s = 0.5
    N, s = p.n_pad, p.s
    ax = (np.arange(N) - N // 2) * s
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    kv = 2 * np.pi * np.array([1, 2, -3]) / (N * s)
    phase = kv[0] * x + kv[1] * y + kv[2] * z
    rho = np.cos(phase)
    phiN, gN = pm.newton_potential(p, rho)
    k2 = (kv * kv).sum()
    assert np.max(np.abs(phiN + 4 * np.pi * p.G * np.cos(phase) / k2)) < 1e-12
    for comp in range(3):
        expect = -(4 * np.pi * p.G / k2) * np.sin(phase) * math.sin(kv[comp] * s) / s
        assert np.max(np.abs(gN[comp] - expect)) < 1e-12


def test_newton_gaussian_field_textbook():
    # One Gaussian of mass M has the textbook potential -G M erf(r/(sqrt2 sigma))/r;
    # g_N is its central difference (the paper's finite-difference gradient),
    # sampled on the axes between 3 sigma and n/8.  The lattice sampling and the
    # periodic images keep the difference within a percent.
    from scipy.special import erf
    p = pm.Params(n=64, n_pad=128, box=64.0, G=1.0, sigma=1.0)
    M = 2.0
    rho = pm.deposit(p, np.array([[0.0, 0.0, 0.0]]), np.array([M]))
    _, gN = pm.newton_potential(p, rho)
    pot = lambda r: -p.G * M * erf(r / math.sqrt(2.0)) / r
    c = p.n_pad // 2
    for r in range(3, 9):
        expect = -(pot(r + 1.0) - pot(r - 1.0)) / 2.0
        assert gN[0, c, c, c + r] == pytest.approx(expect, rel=1e-2)
        assert gN[1, c, c - r, c] == pytest.approx(-expect, rel=1e-2)
        assert gN[2, c + r, c, c] == pytest.approx(expect, rel=1e-2)
        # and the enclosed-mass law within the stencil's O(s^2/r^2) error
        assert abs(gN[0, c, c, c + r]) == pytest.approx(
            M * A.gaussian_enclosed_fraction(r, 1.0) / r ** 2, rel=1.5 / r ** 2)


def _cloud(seed, n, N, mu, **kw):
    w = W.random_cloud(seed, n, N, mu=mu, **kw)
    p = pm.Params.from_dict(w["params"])
    pos = w["pos"].astype(np.float64)
    mass = w["mass"].astype(np.float64)
    return p, pos, mass, pm.deposit(p, pos, mass)


def test_newton_mode_closed_form_any_K():
    # With mu = nu = 1 the iteration reduces to one projection of g_N:
    # phi_hat = At (kt . kappa) phi_hat_N, kappa = sin(k s)/s, for every K >= 1,
    # and H_k = -P_T g_N so r_k = 0 from k = 2 on.
    p, pos, mass, rho = _cloud(2, 16, 40, W.MU_NEWTON, iters=1)
    k, kt = pm.wavevectors(p)
    kx, ky, kz = k[None, None, :], k[None, :, None], k[:, None, None]
    tx, ty, tz = kt[None, None, :], kt[None, :, None], kt[:, None, None]
    k2 = kx ** 2 + ky ** 2 + kz ** 2
    t2 = tx ** 2 + ty ** 2 + tz ** 2
    Ainv = np.where(k2 > 0, 1 / np.where(k2 > 0, k2, 1), 0)
    At = np.where(t2 > 0, 1 / np.where(t2 > 0, t2, 1), 0)
    kap = [np.sin(q * p.s) / p.s for q in (kx, ky, kz)]
    phiNh = -4 * np.pi * p.G * Ainv * np.fft.fftn(rho)
    expect = np.fft.ifftn(At * (tx * kap[0] + ty * kap[1] + tz * kap[2]) * phiNh).real
    for K in (1, 2, 4):
        q = pm.Params.from_dict({**p.__dict__, "iters": K})
        phi, info = pm.aqual_solve(q, rho)
        assert np.max(np.abs(phi - expect)) <= 1e-12 * np.max(np.abs(expect))
        if K >= 3:
            assert info.residuals[0] > 1e-3
            assert max(info.residuals[1:]) < 1e-12


def test_projection_invariants():
    p = pm.Params(n=8, n_pad=16, box=8.0)
    rng = np.random.default_rng(1)
    v = rng.standard_normal((3, 16, 16, 16))
    vh = np.stack([pm.fft3(v[c]) for c in range(3)])
    _, kt = pm.wavevectors(p)
    tx, ty, tz = kt[None, None, :], kt[None, :, None], kt[:, None, None]
    gl, phih = pm.project_curl_free(p, vh)
    ht = pm.project_div_free(p, vh)
    # curl of the curl-free part and divergence of the divergence-free part vanish
    curl = np.stack([ty * gl[2] - tz * gl[1], tz * gl[0] - tx * gl[2], tx * gl[1] - ty * gl[0]])
    assert np.max(np.abs(curl)) < 1e-12 * np.max(np.abs(vh))
    assert np.max(np.abs(tx * ht[0] + ty * ht[1] + tz * ht[2])) < 1e-12 * np.max(np.abs(vh))
    # complementary and idempotent
    assert np.max(np.abs(gl + ht - vh)) < 1e-12 * np.max(np.abs(vh))
    gl2, _ = pm.project_curl_free(p, gl)
    assert np.max(np.abs(gl2 - gl)) < 1e-12 * np.max(np.abs(vh))
    # the field is minus the gradient of phi: g = -i kt phi
    assert np.max(np.abs(gl[0] + 1j * tx * phih)) < 1e-12 * np.max(np.abs(vh))
    # a real field stays real under both projections
    for comp in range(3):
        assert np.max(np.abs(np.fft.ifftn(gl[comp]).imag)) < 1e-13 * np.max(np.abs(v))


def test_interpolation_pair():
    # Sect. 2.1: mu(x) x = y and nu(y) y = x; standard nu as printed; deep pair.
    p = pm.Params(n=8, n_pad=16, box=8.0, a0=2.5, mu=pm.MU_STANDARD)
    y = np.logspace(-6, 6, 61)
    F = np.zeros((3, 61, 1, 1))
    F[0, :, 0, 0] = 0.6 * y * p.a0
    F[2, :, 0, 0] = -0.8 * y * p.a0
    gM = pm.apply_nu(p, F)
    ratio = np.sqrt((gM ** 2).sum(0))[:, 0, 0] / (y * p.a0)
    assert np.allclose(ratio, A.nu_standard_printed(y), rtol=1e-12)
    back = pm.apply_mu(p, gM)
    assert np.allclose(back, F, rtol=1e-12, atol=0)
    x = np.sqrt((gM ** 2).sum(0))[:, 0, 0] / p.a0
    assert np.allclose(A.mu_standard_printed(x) * x, y, rtol=1e-12)
    d = pm.Params(n=8, n_pad=16, box=8.0, a0=2.5, mu=pm.MU_DEEP)
    gd = pm.apply_nu(d, F)
    assert np.allclose(np.sqrt((gd ** 2).sum(0))[:, 0, 0], np.sqrt(y) * p.a0, rtol=1e-12)
    assert np.allclose(pm.apply_mu(d, gd), F, rtol=1e-12)
    # a zero vector maps to zero
    Z = np.zeros((3, 2, 1, 1))
    for q in (p, d):
        assert not np.any(pm.apply_nu(q, Z)) and not np.any(pm.apply_mu(q, Z))


def test_deep_mond_homogeneity():
    # Deep MOND: scaling all masses by lam scales g_M and phi by sqrt(lam);
    # scaling a0 by lam does too.  Exact at every iteration.
    p, pos, mass, rho = _cloud(4, 16, 30, W.MU_DEEP, iters=3)
    phi1, _ = pm.aqual_solve(p, rho)
    phi4, _ = pm.aqual_solve(p, 4.0 * rho)
    assert np.max(np.abs(phi4 - 2.0 * phi1)) <= 1e-11 * np.max(np.abs(phi1))
    q = pm.Params.from_dict({**p.__dict__, "a0": 9.0 * p.a0})
    phi9, _ = pm.aqual_solve(q, rho)
    assert np.max(np.abs(phi9 - 3.0 * phi1)) <= 1e-11 * np.max(np.abs(phi1))


def test_point_mass_deep_mond_field():
    # Sect. 2: an isolated mass has phi = sqrt(G m a0) log r, so |g_M| = sqrt(G m a0)/r.
    # Field from the FD gradient of phi on the grid axes for 3 sigma <= r <= n/8.
    p = pm.Params(n=64, n_pad=128, box=64.0, G=1.0, a0=1e3, mu=pm.MU_DEEP, sigma=1.0)
    rho = pm.deposit(p, np.array([[0.0, 0.0, 0.0]]), np.array([1.0]))
    phi, info = pm.aqual_solve(p, rho, keep_fields=True)
    g = -pm.fd_gradient(p, phi)
    c = p.n_pad // 2
    for r in range(3, 9):
        expect = A.point_mass_field(r, 1.0, p.G, p.a0)
        assert abs(g[0, c, c, c + r]) == pytest.approx(expect, rel=2e-2)
        assert abs(g[1, c, c + r, c]) == pytest.approx(expect, rel=2e-2)
    # spherical field: H stays small (Sect. 2.1, Bekenstein's H = 0)
    H = info.H
    assert math.sqrt((H ** 2).sum()) < 0.05 * math.sqrt((info.gN ** 2).sum())


def test_residual_drops_by_about_ten_per_iteration():
    # Sect. 2.1: the error initially drops by about a factor 10 per iteration.
    p, pos, mass, rho = _cloud(1, 32, 64, W.MU_STANDARD, iters=4)
    _, info = pm.aqual_solve(p, rho)
    r = info.residuals
    assert len(r) == 3
    assert r[1] < r[0] / 5 and r[2] < r[1] / 3


def test_tolerance_mode_exit_rule():
    p, pos, mass, rho = _cloud(1, 16, 30, W.MU_STANDARD, iters=12)
    _, full = pm.aqual_solve(p, rho)
    tol = full.residuals[2] * 1.0001
    q = pm.Params.from_dict({**p.__dict__, "tol": tol})
    _, info = pm.aqual_solve(q, rho)
    # r_3 <= tol is known after iteration 3; the loop exits at iteration 4
    assert info.iterations == 4 and info.converged
    q = pm.Params.from_dict({**p.__dict__, "tol": 1e-30, "iters": 3})
    _, info = pm.aqual_solve(q, rho)
    assert info.iterations == 3 and not info.converged


def test_isothermal_sphere_field():
    # Eq. rho deposited directly on the grid (b = 6 cells, deep MOND); the field
    # strength follows Eq. g with the enclosed mass (spherical symmetry) for
    # 3 <= r <= n/4.  Mass outside the physical region is cut, which does not
    # change the field inside for a spherical distribution.
    p = pm.Params(n=64, n_pad=128, box=64.0, G=1.0, a0=50.0, mu=pm.MU_DEEP)
    N = p.n_pad
    ax = (np.arange(N) - N // 2) * p.s
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    b, M = 6.0, 1.0
    rho = np.where(r < p.n * p.s / 2, A.isothermal_rho(r, M, b), 0.0)
    phi, _ = pm.aqual_solve(p, rho)
    g = -pm.fd_gradient(p, phi)
    c = N // 2
    for rr in (3, 4, 6, 8, 12, 16):
        # central difference of Eq. phi (the paper's FD gradient of the exact
        # potential) and, within the stencil's O(s^2/r^2) error, Eq. g itself
        fd = (A.isothermal_potential(rr + 1, M, b, p.G, p.a0)
              - A.isothermal_potential(rr - 1, M, b, p.G, p.a0)) / 2.0
        assert abs(g[0, c, c, c + rr]) == pytest.approx(fd, rel=2e-2)
        assert abs(g[2, c - rr, c, c]) == pytest.approx(fd, rel=2e-2)
        assert abs(g[1, c, c + rr, c]) == pytest.approx(
            A.isothermal_field(rr, M, b, p.G, p.a0), rel=2e-2 + 0.3 / rr ** 2)


def test_transform_count_is_42(golden, monkeypatch):
    # Sect. 5.2 (iii): the potential takes 42 FFTs, 3 scalar + 13 vector, with
    # four iterations.
    calls = []
    f, fi = pm.fft3, pm.ifft3_real
    monkeypatch.setattr(pm, "fft3", lambda a: calls.append("f") or f(a))
    monkeypatch.setattr(pm, "ifft3_real", lambda a: calls.append("i") or fi(a))
    p, pos, mass, rho = _cloud(1, 8, 10, W.MU_STANDARD, iters=4)
    pm.aqual_solve(p, rho)
    assert len(calls) == golden["ffts_per_step"]["value"]
    assert len(calls) == golden["ffts_per_step"]["scalar"] + 3 * golden["ffts_per_step"]["vector"]


def test_divergence_free_projection_keeps_mean():
    # Reading: the k = 0 mode of H is kept (a constant field is divergence free),
    # so the mean of H after an iteration equals the mean of mu(g_M) g_M.
    p, pos, mass, rho = _cloud(3, 16, 30, W.MU_STANDARD, iters=2)
    _, info = pm.aqual_solve(p, rho, keep_fields=True)
    _, gN = pm.newton_potential(p, rho)
    gM = pm.apply_nu(p, gN)
    gh, _ = pm.project_curl_free(p, np.stack([pm.fft3(gM[c]) for c in range(3)]))
    Fp = pm.apply_mu(p, np.stack([pm.ifft3_real(gh[c]) for c in range(3)]))
    means = info.H.reshape(3, -1).mean(axis=1)
    assert np.allclose(means, Fp.reshape(3, -1).mean(axis=1), rtol=1e-9, atol=1e-18)
    assert np.max(np.abs(means)) > 0.0


def test_start_value_is_taken_divergence_free():
    # H is a curl field (Sect. 2.1): a start value enters through its
    # divergence-free part.  A spectral gradient start i kt psi_hat (kt the
    # wavevector with the Nyquist entry zeroed, built here from its definition)
    # therefore acts like H0 = 0, and restarting from the H of a longer solve
    # continues that solve: its first change equals the change the longer
    # solve would make next.
    p, pos, mass, rho = _cloud(2, 16, 30, W.MU_STANDARD, iters=3)
    phi0, info0 = pm.aqual_solve(p, rho)
    N = p.n_pad
    m = np.fft.fftfreq(N, 1.0 / N)
    kt = np.where(m == -N // 2, 0.0, 2 * np.pi * m / (N * p.s))
    psi_h = np.fft.fftn(np.random.default_rng(5).standard_normal((N, N, N)))
    grads = [kt[None, None, :], kt[None, :, None], kt[:, None, None]]       # x, y, z on [z, y, x]
    H0 = np.stack([np.fft.ifftn(1j * g * psi_h).real for g in grads])
    phi1, info1 = pm.aqual_solve(p, rho, H0=H0 * (np.abs(rho).max() / np.abs(H0).max()))
    assert np.max(np.abs(phi1 - phi0)) < 1e-9 * np.max(np.abs(phi0))
    assert np.allclose(info1.residuals, info0.residuals, rtol=1e-8)

    q6 = pm.Params.from_dict({**p.__dict__, "iters": 6})
    _, long = pm.aqual_solve(q6, rho)
    q4 = pm.Params.from_dict({**p.__dict__, "iters": 4})
    _, mid = pm.aqual_solve(q4, rho, keep_fields=True)
    q3 = pm.Params.from_dict({**p.__dict__, "iters": 3})
    _, rest = pm.aqual_solve(q3, rho, H0=mid.H)
    # mid made residuals r_1..r_3; the restart's r_1, r_2 are the long run's r_4, r_5
    assert np.allclose(rest.residuals, long.residuals[3:5], rtol=1e-7)


def test_qumond_is_the_first_iteration_and_differs_from_aqual():
    # QuMOND's g_M is the curl-free part of nu(|g_N|/a0) g_N: the solve with one
    # evaluation of nu and a zero start computes exactly that.  The two
    # theories agree for a point mass (the field is radial) and differ for a
    # clumpy cloud.
    p, pos, mass, rho = _cloud(5, 16, 40, W.MU_STANDARD, iters=1)
    phi1, _ = pm.aqual_solve(p, rho)
    phiq = pm.qumond_potential(p, rho)
    assert np.max(np.abs(phi1 - phiq)) < 1e-12 * np.max(np.abs(phiq))
    q = pm.Params.from_dict({**p.__dict__, "iters": 12})
    phia, _ = pm.aqual_solve(q, rho)
    d = np.linalg.norm(phia - phiq) / np.linalg.norm(phia)
    assert 1e-4 < d < 5e-2


def test_qumond_point_mass_deep_field():
    # deep MOND: |g_M| = sqrt(G M a0) / r for a point mass in QuMOND as in AQUAL
    p = pm.Params(n=64, n_pad=128, box=64.0, G=1.0, a0=1e3, mu=W.MU_DEEP, sigma=1.0)
    M = 2.0
    rho = pm.deposit(p, np.array([[0.0, 0.0, 0.0]]), np.array([M]))
    phi = pm.qumond_potential(p, rho)
    g = -pm.fd_gradient(p, phi)
    c = p.n_pad // 2
    for r in (4, 6, 8):
        got = abs(g[0, c, c, c + r])
        assert got == pytest.approx(math.sqrt(p.G * M * p.a0) / r, rel=0.03)


def test_apparent_mass_of_a_point_mass_from_gauss_law():
    # Eq. totalmass: the apparent mass inside a sphere is the flux of g_M,
    # R^2 g(R) / G; for a deep-MOND point mass g = sqrt(G M a0)/R, so
    # M_A(<R) = sqrt(G M a0) R / G (the baryonic mass M is a small part of it).
    p = pm.Params(n=64, n_pad=128, box=64.0, G=1.0, a0=1e3, mu=W.MU_DEEP, sigma=1.0, iters=4)
    M = 2.0
    rho = pm.deposit(p, np.array([[0.0, 0.0, 0.0]]), np.array([M]))
    phi, _ = pm.aqual_solve(p, rho)
    rho_a = pm.apparent_density(p, phi)
    N = p.n_pad
    ax = np.arange(N) - N // 2
    z, y, x = np.meshgrid(ax, ax, ax, indexing="ij")
    r = np.sqrt(x * x + y * y + z * z)
    for R in (6, 10, 16):
        assert rho_a[r < R].sum() * p.s ** 3 == pytest.approx(math.sqrt(p.G * M * p.a0) * R / p.G, rel=0.02)


def test_apparent_density_of_the_newton_potential_is_rho():
    # applied to phi_N the operator returns rho (up to the mean, which the
    # periodic potential does not carry) wherever |kt| = |k|, i.e. off the
    # Nyquist planes; the 4-sigma truncation of the kernel leaves content of
    # order 1e-4 there
    p = pm.Params(n=16, n_pad=32, box=16.0, G=0.7, sigma=2.0)
    rho = pm.deposit(p, np.array([[0.3, -0.2, 0.1]]), np.array([1.5]))
    phiN, _ = pm.newton_potential(p, rho)
    rb = pm.apparent_density(p, phiN)
    assert np.max(np.abs(rb - (rho - rho.mean()))) < 2e-4 * np.max(rho)
    # and exactly, mode by mode, off the Nyquist planes
    d = np.fft.fftn(rb - (rho - rho.mean()))
    m = np.fft.fftfreq(32, 1.0 / 32)
    off = (m != -16)
    mask = off[:, None, None] & off[None, :, None] & off[None, None, :]
    assert np.max(np.abs(d[mask])) < 1e-12 * np.max(np.abs(np.fft.fftn(rho)))
