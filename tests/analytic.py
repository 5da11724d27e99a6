"""Closed forms from the paper (and textbook results) used to pin the oracle.

None of these functions shares code with the oracle or the HIP library; each
is written directly from the cited equation.
"""
import math

import numpy as np


def point_mass_field(r, M, G, a0):
    """Deep-MOND field strength of an isolated mass: phi = sqrt(G M a0) log r
    (Sect. 2), so |g| = sqrt(G M a0) / r."""
    return math.sqrt(G * M * a0) / np.asarray(r, dtype=np.float64)


def two_body_force(m1, m2, r, G, a0):
    """Eq. twobodyforce: F12 = 2 sqrt(G a0) / (3 r) (M^1.5 - m1^1.5 - m2^1.5)."""
    M = m1 + m2
    return 2.0 * math.sqrt(G * a0) / (3.0 * r) * (M ** 1.5 - m1 ** 1.5 - m2 ** 1.5)


def two_body_force_rewritten(m1, m2, r, G, a0):
    """Eq. rewrite substituted in Eq. twobodyforce (an algebraically equal form)."""
    M = m1 + m2
    sM = math.sqrt(M)
    return 2.0 * math.sqrt(G * a0) / (3.0 * r) * m1 * m2 * (
        1.0 / (sM + math.sqrt(m1)) + 1.0 / (sM + math.sqrt(m2)))


def two_body_speed(m1, m2, G, a0):
    """Eq. twobodyvelocity: relative speed of the circular two-body orbit."""
    M = m1 + m2
    v2 = 2.0 * math.sqrt(G * M * a0) / 3.0 * (1.0 / (1.0 + math.sqrt(m1 / M))
                                              + 1.0 / (1.0 + math.sqrt(m2 / M)))
    return math.sqrt(v2)


def ring_force(m0, m, n_ring, r2, G, a0):
    """Eq. ringforce: force on one ring particle of an N-gon around m0."""
    M = m0 + n_ring * m
    return 2.0 * math.sqrt(G * a0) / (3.0 * n_ring * r2) * (
        M ** 1.5 - m0 ** 1.5 - n_ring * m ** 1.5)


def ring_speed(m0, m, n_ring, G, a0):
    """Eq. ringvelocity: circular speed of the ring particles."""
    M = m0 + n_ring * m
    q0, q = math.sqrt(m0 / M), math.sqrt(m / M)
    return math.sqrt(2.0 * math.sqrt(G * M * a0) / 3.0 * (1.0 / (1.0 + q0) + q0 - q))


def isothermal_rho(r, M, b):
    """Eq. rho: baryonic density of the deep-MOND isothermal sphere."""
    u = (np.asarray(r, dtype=np.float64) / b) ** 1.5
    return 3.0 * M / (4.0 * math.pi * b ** 3) * (1.0 + u) ** -3


def isothermal_mass(r, M, b):
    """Eq. M: mass inside radius r."""
    r = np.asarray(r, dtype=np.float64)
    u = (r / b) ** 1.5
    return M * r ** 3 / b ** 3 * (1.0 + u) ** -2


def isothermal_potential(r, M, b, G, a0):
    """Eq. phi: phi(r) = (2/3) sqrt(G M a0) log(1 + (r/b)^1.5)."""
    r = np.asarray(r, dtype=np.float64)
    return 2.0 / 3.0 * math.sqrt(G * M * a0) * np.log1p((r / b) ** 1.5)


def isothermal_field(r, M, b, G, a0):
    """Eq. g: field strength sqrt(G M a0 / (b^3 r)) r / (1 + (r/b)^1.5)."""
    r = np.asarray(r, dtype=np.float64)
    return np.sqrt(G * M * a0 / (b ** 3 * r)) * r / (1.0 + (r / b) ** 1.5)


def gaussian_enclosed_fraction(r, sigma):
    """Textbook: mass fraction of an isotropic 3D Gaussian inside radius r."""
    from scipy.special import erf
    r = np.asarray(r, dtype=np.float64)
    return erf(r / (math.sqrt(2.0) * sigma)) - math.sqrt(2.0 / math.pi) * (r / sigma) * np.exp(
        -r * r / (2.0 * sigma * sigma))


def nu_standard_printed(y):
    """The paper's printed inverse of the standard interpolation function,
    nu(y) = sqrt(1/2 + 1/2 sqrt(1 + 4/y^2)) (Sect. 2.1)."""
    y = np.asarray(y, dtype=np.float64)
    return np.sqrt(0.5 + 0.5 * np.sqrt(1.0 + 4.0 / (y * y)))


def mu_standard_printed(x):
    """Eq. mu: mu(x) = x / sqrt(1 + x^2)."""
    x = np.asarray(x, dtype=np.float64)
    return x / np.sqrt(1.0 + x * x)
