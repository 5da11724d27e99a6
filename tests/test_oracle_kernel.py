"""Pins of the oracle's kernel geometry and deposit (Eq. smooth, Sect. 3.1,
appendix 'Fourier transforms')."""
import math

import numpy as np
import pytest

from oracle import pm
import workloads as W


def test_ball_has_251_cells(golden):
    # Sect. 3.1: the ball of radius 4s has 251 pixels.
    assert len(pm.ball_offsets(1.0, 4.0)) == golden["ball_cells_sigma1_radius4"]["value"]


def test_ball_counts_brute_force():
    # Independent count by a triple loop; strict inequality.
    for sigma in (1.0, 1.5, 2.0):
        R = 4.0 * sigma
        cnt = 0
        m = int(R) + 1
        for a in range(-m, m + 1):
            for b in range(-m, m + 1):
                for c in range(-m, m + 1):
                    if a * a + b * b + c * c < R * R:
                        cnt += 1
        assert len(pm.ball_offsets(sigma)) == cnt
    assert [len(pm.ball_offsets(s)) for s in (1.0, 1.5, 2.0)] == [251, 895, 2103]


def _brute_rho(p, pos, mass):
    """rho by looping over every cell and every particle (definition of Eq. smooth
    restricted to the ball around the central pixel, weights normalised)."""
    N = p.n_pad
    s = p.s
    R2 = (p.cutoff * p.sigma) ** 2
    rho = np.zeros((N, N, N))
    for i in range(len(mass)):
        x = pos[i] / s
        c = np.floor(x + 0.5)
        # normaliser: sum over the ball
        norm = 0.0
        cells = []
        for jz in range(N):
            for jy in range(N):
                for jx in range(N):
                    q = np.array([jx, jy, jz], dtype=np.float64) - N // 2
                    # offset from the central pixel, taken on the periodic lattice
                    d = (q - c + N // 2) % N - N // 2
                    if (d * d).sum() < R2:
                        cellpos = c + d
                        w = math.exp(-((cellpos - x) ** 2).sum() / (2 * p.sigma ** 2))
                        norm += w
                        cells.append((jz, jy, jx, w))
        for jz, jy, jx, w in cells:
            rho[jz, jy, jx] += mass[i] * w / norm / s ** 3
    return rho


def test_deposit_matches_brute_force_16():
    rng = np.random.default_rng(3)
    p = pm.Params(n=8, n_pad=16, box=10.0, sigma=1.0)   # s = 1.25
    pos = rng.uniform(-3.0, 3.0, (5, 3))
    pos[4] = [7.4, -7.6, 0.3]                              # ball wraps the box
    mass = rng.uniform(0.5, 2.0, 5)
    rho = pm.deposit(p, pos, mass)
    ref = _brute_rho(p, pos, mass)
    assert np.max(np.abs(rho - ref)) <= 1e-12 * np.max(ref)


def test_deposit_conserves_mass_and_centroid():
    w = W.random_cloud(5, 32, 200, radius_frac=0.25)
    p = pm.Params.from_dict({**w["params"], "box": 24.0})  # s = 0.75
    pos = w["pos"].astype(np.float64)
    mass = w["mass"].astype(np.float64)
    rho = pm.deposit(p, pos, mass)
    assert abs(rho.sum() * p.s ** 3 - mass.sum()) <= 1e-12 * mass.sum()
    ax = (np.arange(p.n_pad) - p.n_pad // 2) * p.s
    cx = (rho.sum(axis=(0, 1)) * ax).sum() * p.s ** 3
    cy = (rho.sum(axis=(0, 2)) * ax).sum() * p.s ** 3
    cz = (rho.sum(axis=(1, 2)) * ax).sum() * p.s ** 3
    ref = (mass[:, None] * pos).sum(axis=0)
    # truncation of the ball makes the kernel centroid differ from x_i by
    # far less than a cell
    assert np.max(np.abs(np.array([cx, cy, cz]) - ref)) / mass.sum() < 1e-3 * p.s


def test_analytic_norm_loses_truncated_tail():
    # Literal prefactor of Eq. smooth: the truncated ball keeps 99.5-99.9 % of
    # the mass for sigma = 1 (the Gaussian's tail beyond 4 sigma).
    p = pm.Params(n=16, n_pad=32, box=16.0, sigma=1.0, flags=pm.F_ANALYTIC_NORM)
    for off in ([0.0, 0.0, 0.0], [0.49, 0.49, 0.49], [0.2, -0.3, 0.1]):
        rho = pm.deposit(p, np.array([off]), np.array([1.0]))
        kept = rho.sum()
        assert 0.994 < kept < 0.9995


def test_gaussian_spectrum_and_nyquist(golden):
    # Appendix 'Fourier transforms': the FT of one particle is
    # m exp(-s^2 k^2 sigma^2 / 2) exp(-i k.r_i), which is exp(-pi^2/2) = .007 at
    # the Nyquist wavevector for sigma = s.  The DFT of the sampled kernel is
    # the periodised spectrum sum_n G(k + 2 pi n / s) (Poisson summation), so at
    # Nyquist it holds the value twice; truncation and normalisation of the
    # ball change it by a few 1e-3 at most.
    assert round(math.exp(-math.pi ** 2 / 2), 3) == golden["gaussian_at_nyquist"]["value"]
    p = pm.Params(n=16, n_pad=32, box=16.0, sigma=1.0)
    rho = pm.deposit(p, np.array([[0.0, 0.0, 0.0]]), np.array([1.0]))
    rh = np.fft.fftn(rho) * p.s ** 3
    k, _ = pm.wavevectors(p)
    m = np.fft.fftfreq(p.n_pad, d=1.0 / p.n_pad)
    # particle at grid index n_pad/2: phase (-1)^m per axis
    for j in range(p.n_pad):
        val = (rh[0, 0, j] * (-1) ** int(m[j])).real
        expect = sum(math.exp(-((k[j] + 2 * math.pi * a / p.s) * p.s * p.sigma) ** 2 / 2.0)
                     for a in range(-3, 4))
        assert abs(val - expect) < 3e-3
    nyq = abs(rh[0, 0, p.n_pad // 2])
    assert nyq == pytest.approx(2 * math.exp(-math.pi ** 2 / 2), abs=3e-3)


def test_out_of_region_flag():
    p = pm.Params(n=32, n_pad=64, box=32.0, sigma=1.0)
    pos = np.array([[0.0, 0.0, 0.0], [12.4, 0.0, 0.0], [12.6, 0.0, 0.0], [0.0, -13.6, 0.0]])
    assert pm.out_of_region(p, pos).tolist() == [False, False, True, True]
