"""FP64 oracle of one particle-mesh step for AQUAL MOND.

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline leg may use this module (see the package docstring).

The oracle follows the paper step by step, with plain full-array NumPy
operations and ``scipy.fft`` complex-to-complex transforms (taking the real
part after every inverse).  Readings of points the paper leaves open are
marked "Reading:" where they are used.

Conventions
-----------
* Grid arrays are indexed ``[z, y, x]`` (x fastest in memory); the FFT box has
  ``n_pad`` cells per axis of width ``s = box / n``; grid index j on an axis is
  the point (j - n_pad/2) s (appendix "Fourier transforms", with n -> n_pad).
* Positions are ``[N, 3]`` as (x, y, z) measured from the box centre.
* Vector fields are ``[3, n_pad, n_pad, n_pad]`` with components (x, y, z).
"""
from __future__ import annotations

import math
import os
from dataclasses import dataclass, field

import numpy as np
import scipy.fft as sfft

MU_STANDARD, MU_DEEP, MU_NEWTON = 0, 1, 2
F_ANALYTIC_NORM = 1

WORKERS = int(os.environ.get("ORACLE_FFT_WORKERS", os.cpu_count() or 1))


@dataclass
class Params:
    """Statement of the problem (Sect. 2 and 3 of the paper).

    n, n_pad : physical cells per axis and FFT box per axis (n_pad = 2n gives
               the empty margin around the matter that Sect. 3 asks for).
    box      : side of the physical n-grid; the pixel width is s = box / n.
    G, a0    : Newton's constant and Milgrom's acceleration (Eq. PDE).
    mu       : interpolation function: standard x/sqrt(1+x^2) (Eq. mu),
               deep MOND mu(x)=x (Sect. 4) or Newton mu=1 (the high-field limit).
    sigma    : Gaussian kernel standard deviation in cells (paper: 1).
    cutoff   : ball radius in units of sigma (paper: 4, giving 251 cells).
    iters    : K, the number of evaluations of nu (paper: 4).
    tol      : 0 runs exactly K iterations; > 0 stops once the residual of the
               previous iteration is <= tol (K is then the maximum).
    flags    : F_ANALYTIC_NORM uses the literal Gaussian prefactor instead of
               normalising by the ball sum.
    """
    n: int
    n_pad: int
    box: float
    G: float = 1.0
    a0: float = 1.0
    mu: int = MU_STANDARD
    sigma: float = 1.0
    cutoff: float = 4.0
    iters: int = 4
    tol: float = 0.0
    flags: int = 0

    @property
    def s(self) -> float:
        return self.box / self.n

    @classmethod
    def from_dict(cls, d):
        keys = cls.__dataclass_fields__.keys()
        return cls(**{k: v for k, v in d.items() if k in keys})


# ---------------------------------------------------------------------------
# Kernel geometry (Sect. 3.1, Fig. 1 and the initialisation of the flow scheme)
# ---------------------------------------------------------------------------

def ball_offsets(sigma: float, cutoff: float = 4.0) -> np.ndarray:
    """Integer offsets d with |d| < cutoff * sigma, measured from the central pixel.

    Reading: the ball is strict (|d|^2 < R^2).  With sigma = 1 and cutoff = 4
    this is the paper's list of 251 cells (Sect. 3.1); the non-strict ball
    would have 257.
    """
    R = cutoff * sigma
    m = int(math.floor(R))
    r = np.arange(-m, m + 1)
    dz, dy, dx = np.meshgrid(r, r, r, indexing="ij")
    d = np.stack([dx.ravel(), dy.ravel(), dz.ravel()], axis=1)
    keep = (d * d).sum(axis=1) < R * R
    return d[keep].astype(np.int64)


def central_pixel(pos_cells: np.ndarray) -> np.ndarray:
    """Pixel containing the particle: nearest grid point, ties rounded up."""
    return np.floor(pos_cells + 0.5).astype(np.int64)


def kernel_weights(p: Params, pos: np.ndarray, ball: np.ndarray | None = None):
    """Grid indices and normalised Gaussian weights of each particle's ball.

    Eq. smooth: a particle at r_i contributes exp(-|r - r_i|^2 / (2 sigma^2 s^2))
    to the pixels of its ball.  Reading: by default the weights are divided by
    their sum over the ball (so the truncated kernel keeps the mass exactly);
    with F_ANALYTIC_NORM the literal prefactor 1 / ((2 pi)^(3/2) sigma^3) is used.

    Returns (idx [N, B, 3] int64 grid indices (x, y, z) in [0, n_pad), w [N, B]).
    """
    if ball is None:
        ball = ball_offsets(p.sigma, p.cutoff)
    x = np.asarray(pos, dtype=np.float64) / p.s
    c = central_pixel(x)
    cells = c[:, None, :] + ball[None, :, :]
    delta = cells - x[:, None, :]
    w = np.exp(-(delta * delta).sum(axis=2) / (2.0 * p.sigma * p.sigma))
    if p.flags & F_ANALYTIC_NORM:
        w = w / ((2.0 * math.pi) ** 1.5 * p.sigma ** 3)
    else:
        w = w / w.sum(axis=1, keepdims=True)
    idx = np.mod(cells + p.n_pad // 2, p.n_pad)
    return idx, w


def out_of_region(p: Params, pos: np.ndarray) -> np.ndarray:
    """Particles whose ball leaves the physical n^3 region (Sect. 3: matter must
    stay away from the boundary).  Such particles are still computed, with grid
    indices wrapped modulo n_pad."""
    m = int(math.ceil(p.cutoff * p.sigma)) - 1      # largest |d_axis| in the ball
    c = central_pixel(np.asarray(pos, dtype=np.float64) / p.s)
    lo, hi = -p.n // 2, p.n // 2 - 1
    return np.any((c - m < lo) | (c + m > hi), axis=1)


# ---------------------------------------------------------------------------
# Deposit (Eq. smooth; flow scheme main loop, step 2)
# ---------------------------------------------------------------------------

def deposit(p: Params, pos: np.ndarray, mass: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """Mass density rho_B on the n_pad^3 grid from the Gaussian kernel (Eq. smooth).

    rho[c_i + d] += m_i w_id / s^3 for every particle i and ball offset d.
    """
    N = p.n_pad
    ball = ball_offsets(p.sigma, p.cutoff)
    rho = np.zeros(N ** 3)
    mass = np.asarray(mass, dtype=np.float64)
    for a in range(0, len(mass), chunk):
        idx, w = kernel_weights(p, pos[a:a + chunk], ball)
        flat = (idx[..., 2] * N + idx[..., 1]) * N + idx[..., 0]
        rho += np.bincount(flat.ravel(), weights=(mass[a:a + chunk, None] * w).ravel() / p.s ** 3,
                           minlength=N ** 3)
    return rho.reshape(N, N, N)


# ---------------------------------------------------------------------------
# Spectral operators (appendix "Fourier transforms" and the flow scheme)
# ---------------------------------------------------------------------------

def wavevectors(p: Params):
    """Per-axis wavevector k = 2 pi m / (n_pad s), m in fftfreq order.

    Returns (k, kt): the true k, and k with the Nyquist entry m = -n_pad/2 set
    to zero.  Reading: the curl-free and divergence-free projections use kt
    (the Nyquist wavevector of an odd operator is zero on a real periodic
    lattice); the Newton inverse Laplacian keeps the true |k|^2.
    """
    N = p.n_pad
    m = np.fft.fftfreq(N, d=1.0 / N)
    k = 2.0 * math.pi * m / (N * p.s)
    kt = np.where(m == -N // 2, 0.0, k)
    return k, kt


def _grids(k):
    return k[None, None, :], k[None, :, None], k[:, None, None]   # kx, ky, kz


def fft3(a):
    return sfft.fftn(a, workers=WORKERS)


def ifft3_real(a):
    return sfft.ifftn(a, workers=WORKERS).real


def fd_gradient(p: Params, phi: np.ndarray) -> np.ndarray:
    """Periodic second-order central differences, (phi(j+1) - phi(j-1)) / (2s).

    Reading: the paper says only "finite differences"; the central stencil is
    the simplest antisymmetric one (Sect. 3.2, Sect. 5.1).
    """
    out = np.empty((3,) + phi.shape)
    for comp, axis in ((0, 2), (1, 1), (2, 0)):
        out[comp] = (np.roll(phi, -1, axis=axis) - np.roll(phi, 1, axis=axis)) / (2.0 * p.s)
    return out


def newton_potential(p: Params, rho: np.ndarray):
    """phi_N and g_N from rho (flow scheme main loop, steps 3-6).

    phi_hat_N = -4 pi G A rho_hat with A = 1/(k.k), A(0) = 0; g_N = -D phi_N.
    Reading: the flow scheme prints +4 pi G A rho_hat; with g_N = -grad phi_N
    and div g_N = -4 pi G rho (Eq. newtongrav) the sign must be negative.
    """
    k, _ = wavevectors(p)
    kx, ky, kz = _grids(k)
    k2 = kx * kx + ky * ky + kz * kz
    A = np.where(k2 > 0.0, 1.0 / np.where(k2 > 0.0, k2, 1.0), 0.0)
    phiN = ifft3_real(-4.0 * math.pi * p.G * A * fft3(rho))
    gN = -fd_gradient(p, phiN)
    return phiN, gN


def project_curl_free(p: Params, gh: np.ndarray):
    """Curl-free part in Fourier space (Eq. rotg; flow scheme iteration steps 3-4).

    phi_hat = i At (kt . g_hat) and g_hat <- -i kt phi_hat = kt At (kt . g_hat),
    with At = 1/|kt|^2 (0 where kt = 0).  Returns (g_hat_projected, phi_hat).
    """
    _, kt = wavevectors(p)
    kx, ky, kz = _grids(kt)
    k2 = kx * kx + ky * ky + kz * kz
    At = np.where(k2 > 0.0, 1.0 / np.where(k2 > 0.0, k2, 1.0), 0.0)
    dot = kx * gh[0] + ky * gh[1] + kz * gh[2]
    phih = 1j * At * dot
    out = np.stack([-1j * kx * phih, -1j * ky * phih, -1j * kz * phih])
    return out, phih


def project_div_free(p: Params, Hh: np.ndarray) -> np.ndarray:
    """Divergence-free part (Eq. divH; flow scheme iteration step "make the field
    divergence free"): H_hat <- H_hat - kt At (kt . H_hat).  The k = 0 mode is
    kept (Reading: a constant field is divergence free)."""
    _, kt = wavevectors(p)
    kx, ky, kz = _grids(kt)
    k2 = kx * kx + ky * ky + kz * kz
    At = np.where(k2 > 0.0, 1.0 / np.where(k2 > 0.0, k2, 1.0), 0.0)
    dot = kx * Hh[0] + ky * Hh[1] + kz * Hh[2]
    return np.stack([Hh[0] - kx * At * dot, Hh[1] - ky * At * dot, Hh[2] - kz * At * dot])


# ---------------------------------------------------------------------------
# The algebraic equations (Eqs. inverse and interpolation)
# ---------------------------------------------------------------------------

def apply_nu(p: Params, F: np.ndarray) -> np.ndarray:
    """g_M = nu(|F|/a0) F (Eq. inverse).

    Standard pair (Eq. mu and the nu printed after it): with y = |F|/a0 the
    strength is |g_M| = a0 x with x = sqrt((y/2)(y + sqrt(y^2 + 4))), the same
    number as nu(y) y but without forming 4/y^2.  Deep MOND: nu(y) = 1/sqrt(y),
    so g_M = F sqrt(a0/|F|).  Newton: nu = 1.  A zero vector maps to zero.
    """
    if p.mu == MU_NEWTON:
        return F.copy()
    Fm = np.sqrt((F * F).sum(axis=0))
    safe = np.where(Fm > 0.0, Fm, 1.0)
    if p.mu == MU_DEEP:
        ratio = np.sqrt(p.a0 / safe)
    else:
        y = safe / p.a0
        x = np.sqrt(0.5 * y * (y + np.sqrt(y * y + 4.0)))
        ratio = x / y
    return F * np.where(Fm > 0.0, ratio, 0.0)


def apply_mu(p: Params, gM: np.ndarray) -> np.ndarray:
    """F = mu(|g_M|/a0) g_M (Eq. interpolation).

    Standard: mu(x) = x / sqrt(1 + x^2) (Eq. mu); deep MOND: mu(x) = x
    (Sect. 4); Newton: mu = 1.
    """
    if p.mu == MU_NEWTON:
        return gM.copy()
    x = np.sqrt((gM * gM).sum(axis=0)) / p.a0
    if p.mu == MU_DEEP:
        m = x
    else:
        m = x / np.sqrt(1.0 + x * x)
    return gM * m


# ---------------------------------------------------------------------------
# The AQUAL solve (Sect. 2.1 iteration; flow scheme main loop, steps 3-9)
# ---------------------------------------------------------------------------

@dataclass
class SolveInfo:
    iterations: int = 0
    residuals: list = field(default_factory=list)   # r_k for k = 1, 2, ...
    converged: bool = True
    H: np.ndarray | None = None                     # last H (real space)
    gN: np.ndarray | None = None


def aqual_solve(p: Params, rho: np.ndarray, H0: np.ndarray | None = None,
                keep_fields: bool = False):
    """Potential phi of Eq. PDE from rho by the fixed-point iteration of Sect. 2.1.

    g_N is solved once and stored; H starts at the divergence-free part of H0
    (zero by default; H is a curl field in the decomposition of Sect. 2.1, so
    a start value is projected like every later iterate).  Each
    iteration: F = g_N + H; g_M = nu(F) F; project g_M curl-free in Fourier
    space (giving phi_hat); stop at the K-th evaluation of nu (the flow scheme
    exits after the projection of the fourth iteration); otherwise
    F' = mu(g_M) g_M; H = F' - g_N projected divergence-free; repeat.

    Reading of the residual (the paper estimates the error from the change of
    H): r_k = ||H_k - H_{k-1}|| / ||g_N|| over the whole box.  With tol > 0 the
    loop stops at iteration k once r_{k-1} <= tol.
    """
    _, gN = newton_potential(p, rho)
    if H0 is None:
        H = np.zeros_like(gN)
    else:
        H0 = np.asarray(H0, dtype=np.float64)
        H = np.stack([ifft3_real(c) for c in project_div_free(p, np.stack([fft3(H0[c]) for c in range(3)]))])
    norm_gN = math.sqrt(float((gN * gN).sum()))
    info = SolveInfo()
    K = max(int(p.iters), 1)
    F = gN + H
    phih = None
    for k in range(1, K + 1):
        gM = apply_nu(p, F)
        gh = np.stack([fft3(gM[c]) for c in range(3)])
        gh, phih = project_curl_free(p, gh)
        info.iterations = k
        if k == K:
            break
        if p.tol > 0.0 and info.residuals and info.residuals[-1] <= p.tol:
            break
        gM = np.stack([ifft3_real(gh[c]) for c in range(3)])
        Fp = apply_mu(p, gM)
        Ht = Fp - gN
        Hh = project_div_free(p, np.stack([fft3(Ht[c]) for c in range(3)]))
        Hn = np.stack([ifft3_real(Hh[c]) for c in range(3)])
        dH = Hn - H
        info.residuals.append(math.sqrt(float((dH * dH).sum())) / norm_gN if norm_gN > 0 else 0.0)
        H = Hn
        F = gN + H
    if p.tol > 0.0:
        info.converged = bool(info.residuals and info.residuals[-1] <= p.tol)
    phi = ifft3_real(phih)
    if keep_fields:
        info.H = H
        info.gN = gN
    return phi, info


def external_field_density(p: Params, g_ext) -> np.ndarray:
    """Density of the external-field sheets (Sect. 5: a permanent dipolar mass
    layer on the plane farthest from the particles, a pixel layer of mass M
    beside one of mass -M).

    Reading: one sheet pair per axis d, +rho_d in every cell of plane
    n_pad - 1 and -rho_d in every cell of plane 0 (the two planes straddle the
    periodic boundary, the farthest from matter at the centre), with
    rho_d = g_d L / (4 pi G s^2), L = n_pad s.  The Newton field of a periodic
    sheet pair has zero mean over the period and jumps by 4 pi G rho_d s
    across the pair, so in the bulk it is uniform, g_d, pointing from the
    positive to the negative sheet.
    """
    N = p.n_pad
    L = N * p.s
    out = np.zeros((N, N, N))
    for d, axis in ((0, 2), (1, 1), (2, 0)):          # x, y, z components; arrays are [z][y][x]
        rd = float(g_ext[d]) * L / (4.0 * math.pi * p.G * p.s * p.s)
        if rd == 0.0:
            continue
        hi = [slice(None)] * 3
        lo = [slice(None)] * 3
        hi[axis] = N - 1
        lo[axis] = 0
        out[tuple(hi)] += rd
        out[tuple(lo)] -= rd
    return out


def qumond_potential(p: Params, rho: np.ndarray) -> np.ndarray:
    """Potential of quasi-linear MOND (Sect. 2, the equivalent system for
    QuMOND): g_M + H = nu(|g_N|/a0) g_N with g_M curl-free and H divergence
    free, so g_M is the curl-free part of nu(|g_N|/a0) g_N and phi its
    potential.  No iteration is involved."""
    _, gN = newton_potential(p, rho)
    rhs = apply_nu(p, gN)
    _, phih = project_curl_free(p, np.stack([fft3(rhs[c]) for c in range(3)]))
    return ifft3_real(phih)


def apparent_density(p: Params, phi: np.ndarray) -> np.ndarray:
    """Apparent density of Eq. apparentdensity, rho_A = -div(g)/(4 pi G) with
    g = -grad phi, written with the same discrete wavevector kt as the
    projections (the field g_M of the solve is -i kt phi_hat):
    rho_A_hat = -|kt|^2 phi_hat / (4 pi G).  The k = 0 mode is zero: a
    potential on the periodic box does not fix the mean density.  Applied to
    the Newton potential it gives the baryonic density the same way, and
    the difference of the two is the phantom density."""
    _, kt = wavevectors(p)
    kx, ky, kz = _grids(kt)
    k2 = kx * kx + ky * ky + kz * kz
    return ifft3_real(-k2 * fft3(phi) / (4.0 * math.pi * p.G))


# ---------------------------------------------------------------------------
# Forces and time integration (Eq. gi, Eq. motion; flow scheme steps 10-11)
# ---------------------------------------------------------------------------

def smooth_accel(p: Params, phi: np.ndarray, pos: np.ndarray, chunk: int = 8192) -> np.ndarray:
    """Kernel-smoothed acceleration of each particle (Eq. gi).

    g_i = - sum_d w_id (D phi)(c_i + d), with D the finite-difference gradient
    and w the same normalised Gaussian weights as the deposit.
    """
    Dphi = fd_gradient(p, phi)
    ball = ball_offsets(p.sigma, p.cutoff)
    acc = np.empty((len(pos), 3))
    for a in range(0, len(pos), chunk):
        idx, w = kernel_weights(p, pos[a:a + chunk], ball)
        for comp in range(3):
            vals = Dphi[comp][idx[..., 2], idx[..., 1], idx[..., 0]]
            acc[a:a + chunk, comp] = -(w * vals).sum(axis=1)
    return acc


def interp_push(p: Params, phi, pos, vel, dt_kick: float, dt_drift: float):
    """Leapfrog kick then drift (Eq. motion): v <- v + g dt_kick; r <- r + v dt_drift."""
    acc = smooth_accel(p, phi, pos)
    vel = np.asarray(vel, dtype=np.float64) + acc * dt_kick
    pos = np.asarray(pos, dtype=np.float64) + vel * dt_drift
    return pos, vel


def pm_step(p: Params, pos, vel, mass, dt: float, H0=None, g_ext=None):
    """One PM step: deposit(r) -> solve -> kick(dt) -> drift(dt).

    Reading: positions and velocities are half a step apart (Sect. 3); one step
    evaluates the force at the current positions, kicks by dt and drifts by dt,
    which is the alternation of the flow scheme with one fixed phase.  g_ext:
    optional uniform external Newtonian field, added as the sheets of
    external_field_density.
    """
    rho = deposit(p, pos, mass)
    if g_ext is not None:
        rho = rho + external_field_density(p, g_ext)
    phi, info = aqual_solve(p, rho, H0)
    pos, vel = interp_push(p, phi, pos, vel, dt, dt)
    return pos, vel, info


# ---------------------------------------------------------------------------
# Diagnostics (constants of motion, Sect. 4.1; energies, Sect. 4.3)
# ---------------------------------------------------------------------------

def potential_at_particles(p: Params, phi, pos) -> np.ndarray:
    """phi smoothed with the particle kernel: sum_d w_id phi(c_i + d)."""
    idx, w = kernel_weights(p, pos)
    return (w * phi[idx[..., 2], idx[..., 1], idx[..., 0]]).sum(axis=1)


def diagnostics(p: Params, pos, vel, mass, phi=None) -> dict:
    """Total momentum P, angular momentum L, kinetic energy, sum m_i phi_i, mass."""
    pos = np.asarray(pos, np.float64)
    vel = np.asarray(vel, np.float64)
    mass = np.asarray(mass, np.float64)
    out = dict(P=(mass[:, None] * vel).sum(axis=0),
               L=(mass[:, None] * np.cross(pos, vel)).sum(axis=0),
               Ekin=0.5 * float((mass * (vel * vel).sum(axis=1)).sum()),
               mass=float(mass.sum()))
    if phi is not None:
        out["Epot_sum"] = float((mass * potential_at_particles(p, phi, pos)).sum())
    return out
