"""Pins of the external field made by a dipole sheet (Sect. 5) in the FP64
oracle.

Closed forms used:
- Newton mode: a periodic sheet pair of +-rho_c gives the bulk the uniform
  field 4 pi G rho_c s^2 / L, since the field has zero mean over the period
  and jumps by 4 pi G rho_c s across the pair.
- MOND, standard mu: the bulk field is again the sheets' field, up to
  O(s/L).  Periodicity fixes the potential drop across the box, and the
  fields inside the sheet gap are Newtonian-strong.
- External field effect: linearising AQUAL (Sect. 2) about a uniform field
  g_e along e gives mu_e [lap psi + L_e d_e^2 psi] = 4 pi G rho, with
  mu_e = mu(g_e / a0) and L_e = d ln mu / d ln x at g_e / a0 (for the
  standard mu, L_e = 1 / (1 + x^2)).  Stretching the e axis by
  sqrt(1 + L_e) turns this into Poisson's equation, so a point mass m has
  psi = -G m / (mu_e sqrt(1 + L_e) sqrt(rho_perp^2 + z_e^2 / (1 + L_e))).
  Its field is G m / (mu_e r^2) along e and G m / (mu_e sqrt(1 + L_e) r^2)
  across it.
"""
import math

import numpy as np
import pytest

from oracle import pm as orc
import workloads as W
from tests.gpu_util import oparams


def _centre(a, N, h=8):
    c = slice(N // 2 - h, N // 2 + h)
    return a[..., c, c, c]


@pytest.mark.parametrize("g", [(0.3, -0.2, 0.1), (0.0, 0.0, 1.0), (-2.0, 0.0, 0.0)])
def test_sheets_give_a_uniform_newton_field(g):
    p = oparams(W.params(32, G=1.0, a0=1.0, mu=2, iters=1))
    N = p.n_pad
    sheets = orc.external_field_density(p, g)
    assert abs(sheets.sum()) < 1e-9 * np.abs(sheets).sum()          # a dipole layer: no net mass
    _, gN = orc.newton_potential(p, sheets)
    bulk = _centre(gN, N)
    gn = np.linalg.norm(g)
    for d in range(3):
        assert np.max(np.abs(bulk[d] - g[d])) < 5e-4 * gn
    # the Newton-mode solve returns the same field (mu = nu = 1)
    phi, _ = orc.aqual_solve(p, sheets)
    gM = _centre(-orc.fd_gradient(p, phi), N)
    for d in range(3):
        assert np.max(np.abs(gM[d] - g[d])) < 5e-4 * gn


def test_mond_bulk_field_is_the_sheets_field():
    g = np.array([0.0, 0.6, 0.8])
    errs = []
    for n in (32, 48):
        p = oparams(W.params(n, G=1.0, a0=1.0, mu=0, iters=12))
        phi, info = orc.aqual_solve(p, orc.external_field_density(p, g))
        bulk = _centre(-orc.fd_gradient(p, phi), p.n_pad)
        mean = bulk.reshape(3, -1).mean(axis=1)
        assert np.max(np.abs(bulk - mean[:, None, None, None])) < 2e-3      # uniform
        # along g (each axis's sheets carry their own O(s / L) excess, so the
        # direction is off by ~1e-3), about |g|, far from nu(|g| / a0) |g| = 1.27 |g|
        assert np.linalg.norm(np.cross(mean, g)) < 5e-3 * np.linalg.norm(mean) * np.linalg.norm(g)
        errs.append(np.linalg.norm(mean) / np.linalg.norm(g) - 1.0)
    assert 0.0 < errs[1] < errs[0] < 0.03          # an O(s / L) excess that shrinks with the box


@pytest.mark.parametrize("axis", [0, 2])
def test_external_field_effect_matches_linearised_aqual(axis):
    n, m = 32, 0.1
    p = oparams(W.params(n, G=1.0, a0=1.0, mu=0, iters=40))
    N, c = p.n_pad, p.n_pad // 2
    g = np.zeros(3)
    g[axis] = 1.0
    sheets = orc.external_field_density(p, g)
    phi0, _ = orc.aqual_solve(p, sheets)
    phi1, info = orc.aqual_solve(p, sheets + orc.deposit(p, np.zeros((1, 3)), np.array([m])))
    assert info.residuals[-1] < 1e-10
    g0 = -orc.fd_gradient(p, phi0)
    dg = -orc.fd_gradient(p, phi1) - g0                  # the mass's own field
    x = abs(g0[axis][c, c, c]) / p.a0                     # local external MOND field
    mu_e = x / math.sqrt(1.0 + x * x)
    L_e = 1.0 / (1.0 + x * x)
    other = 2 if axis == 0 else 0
    for r in (8, 10):
        at_par = [c, c, c]
        at_par[2 - axis] += r                             # arrays are [z][y][x]
        at_perp = [c, c, c]
        at_perp[2 - other] += r
        par = -dg[axis][tuple(at_par)]                    # points back to the mass
        perp = -dg[other][tuple(at_perp)]
        exp_par = p.G * m / (mu_e * r * r)
        exp_perp = exp_par / math.sqrt(1.0 + L_e)
        assert par == pytest.approx(exp_par, rel=0.06)
        assert perp == pytest.approx(exp_perp, rel=0.03)
        assert perp / par == pytest.approx(1.0 / math.sqrt(1.0 + L_e), rel=0.05)
        # without the external field the field would be deep MOND, sqrt(G m a0) / r
        assert par < 0.2 * math.sqrt(p.G * m * p.a0) / r
