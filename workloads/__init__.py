"""Seeded synthetic workloads for the MOND particle-mesh step.

This module only draws inputs: particle positions, velocities and masses plus
the run parameters of each workload.  It holds none of the method's arithmetic
(no deposit, no field solve, no force), so that the FP64 oracle and the HIP
path can both take their inputs from here without sharing any computation.

Every generator works in FP64 with ``numpy.random.default_rng(seed)`` (PCG64)
and casts once to FP32; the FP32 arrays are the canonical inputs.  A caller
that needs FP64 (the oracle) promotes these FP32 values.

Conventions: lengths are in units of the pixel width ``s = box / n``; the
origin is the centre of the FFT box; positions are ``[N, 3]`` as (x, y, z).
The parameter dictionaries use the names of the C parameter block
(n, n_pad, box, G, a0, mu, sigma, cutoff, iters, tol, flags).
"""
from __future__ import annotations

import math

import numpy as np

MU_STANDARD, MU_DEEP, MU_NEWTON = 0, 1, 2


def params(n, n_pad=None, box=None, G=1.0, a0=1.0, mu=MU_STANDARD, sigma=1.0,
           cutoff=4.0, iters=4, tol=0.0, flags=0):
    """Parameter dictionary with the defaults of the paper's scheme.

    n_pad defaults to 2n (empty margin around the matter, Sect. 3 of the
    paper); box defaults to n so that the pixel width s is 1.
    """
    return dict(n=int(n), n_pad=int(n_pad if n_pad is not None else 2 * n),
                box=float(box if box is not None else n), G=float(G), a0=float(a0),
                mu=int(mu), sigma=float(sigma), cutoff=float(cutoff),
                iters=int(iters), tol=float(tol), flags=int(flags))


def _f32(*arrays):
    return tuple(np.ascontiguousarray(a, dtype=np.float32) for a in arrays)


def ring_speed(m0, m_ring_total, n_ring, G, a0):
    """Circular speed of an N-gon ring around a central mass in deep MOND.

    Eq. ringvelocity (Sect. 4.2): v^2 = (2/3) sqrt(G M a0) *
    (1/(1+sqrt(m0/M)) + sqrt(m0/M) - sqrt(m/M)), with M = m0 + N m.
    Used only to set the initial velocities of the ring workload.
    """
    M = m0 + m_ring_total
    m = m_ring_total / n_ring
    q0, q = math.sqrt(m0 / M), math.sqrt(m / M)
    return math.sqrt(2.0 / 3.0 * math.sqrt(G * M * a0) * (1.0 / (1.0 + q0) + q0 - q))


def two_body(shift=(0.0, 0.0, 0.0)):
    """Deep-MOND two-body case: 64^3 grid in a 128^3 periodic FFT box.

    m1 = 1.0 and m2 = 0.5 at rest, 8 cells apart on the x axis with the
    centre of mass at the origin (plus an optional shift, in cells).  G = 1,
    a0 = 1e3, deep-MOND interpolation, Gaussian sigma = 2 cells, 4 iterations,
    dt = 0.01 for 200 steps (Sect. 4.1 of the paper).
    """
    p = params(64, a0=1e3, mu=MU_DEEP, sigma=2.0)
    sh = np.asarray(shift, dtype=np.float64)
    pos = np.array([[-8.0 / 3.0, 0.0, 0.0], [16.0 / 3.0, 0.0, 0.0]]) + sh
    vel = np.zeros((2, 3))
    mass = np.array([1.0, 0.5])
    pos, vel, mass = _f32(pos, vel, mass)
    return dict(params=p, pos=pos, vel=vel, mass=mass, dt=0.01, steps=200,
                workload="two_body_64")


def ring(seed=0, n_ring=4096, radius=20.0, n=128, sigma=1.5, jitter=0.1):
    """Central mass plus a rotating ring of equal test particles (Sect. 4.2).

    M0 = 1 at the origin; n_ring particles with total mass 1e-3 on a circle of
    the given radius (cells) in the xy plane, each radius jittered by
    N(0, jitter^2) cells; tangential speed from Eq. ringvelocity.  G = 1,
    a0 = 1e3, deep-MOND interpolation, dt = 0.02.
    """
    rng = np.random.default_rng(seed)
    G, a0, m0, mr = 1.0, 1e3, 1.0, 1e-3
    p = params(n, a0=a0, mu=MU_DEEP, sigma=sigma)
    th = 2.0 * np.pi * np.arange(n_ring) / n_ring
    r = radius + jitter * rng.standard_normal(n_ring)
    v = ring_speed(m0, mr, n_ring, G, a0)
    pos = np.zeros((n_ring + 1, 3))
    vel = np.zeros((n_ring + 1, 3))
    pos[1:, 0], pos[1:, 1] = r * np.cos(th), r * np.sin(th)
    vel[1:, 0], vel[1:, 1] = -v * np.sin(th), v * np.cos(th)
    mass = np.concatenate([[m0], np.full(n_ring, mr / n_ring)])
    pos, vel, mass = _f32(pos, vel, mass)
    return dict(params=p, pos=pos, vel=vel, mass=mass, dt=0.02, steps=1000,
                ring_speed=v, workload=f"ring_{n}")


def isothermal_positions(rng, count, b, r_max):
    """Radii and directions from Eq. boxmuller (Sect. 4.3), rejecting r > r_max."""
    out = np.empty((0, 3))
    while out.shape[0] < count:
        k = count - out.shape[0]
        xi = rng.uniform(-1.0, 1.0, k)
        eta = rng.uniform(0.0, 1.0, k)
        zeta = rng.uniform(0.0, 2.0 * np.pi, k)
        eta = np.clip(eta, 1e-300, 1.0 - 1e-16)
        rad = b * (1.0 / np.sqrt(eta) - 1.0) ** (-2.0 / 3.0)
        st = np.sqrt(1.0 - xi * xi)
        x = np.stack([st * np.cos(zeta), st * np.sin(zeta), xi], axis=1) * rad[:, None]
        out = np.concatenate([out, x[rad <= r_max]], axis=0)
    return out[:count]


def maxwellian(rng, count, v2mean):
    """Velocities of Eq. boxmuller: each Cartesian component ~ N(0, <v^2>/3)."""
    eta2 = 1.0 - rng.uniform(0.0, 1.0, count)
    eta3 = 1.0 - rng.uniform(0.0, 1.0, count)
    z2 = rng.uniform(0.0, 2.0 * np.pi, count)
    z3 = rng.uniform(0.0, 2.0 * np.pi, count)
    a = np.sqrt(-2.0 / 3.0 * v2mean * np.log(eta2))
    c = np.sqrt(-2.0 / 3.0 * v2mean * np.log(eta3))
    return np.stack([a * np.cos(z2), a * np.sin(z2), c * np.cos(z3)], axis=1)


def isothermal_sphere(seed=0, N=1 << 20, n=256, b=16.0, r_max=120.0, M=1.0, G=1.0):
    """Self-consistent isothermal sphere, the throughput workload.

    N equal masses (total M) drawn from Eq. boxmuller with length b; the
    Maxwellian dispersion is <v^2> = (2/3) sqrt(G M a0) (Eq. vsqsuare).  a0 is
    set so that the Newtonian field at the half-mass radius
    r_h = b / (sqrt(2) - 1)^(2/3) equals a0, putting the outer half of the
    mass in the deep-MOND regime; standard interpolation, sigma = 1 cell,
    4 iterations, dt = 0.1 s / sqrt(<v^2>).
    """
    rng = np.random.default_rng(seed)
    r_h = b / (math.sqrt(2.0) - 1.0) ** (2.0 / 3.0)
    a0 = G * M / (2.0 * r_h * r_h)
    v2 = 2.0 / 3.0 * math.sqrt(G * M * a0)
    p = params(n, a0=a0, mu=MU_STANDARD, sigma=1.0, G=G)
    pos = isothermal_positions(rng, N, b, r_max)
    vel = maxwellian(rng, N, v2)
    mass = np.full(N, M / N)
    pos, vel, mass = _f32(pos, vel, mass)
    return dict(params=p, pos=pos, vel=vel, mass=mass, dt=0.1 / math.sqrt(v2),
                steps=100, v2mean=v2, b=b, workload=f"isothermal_{n}_N{N}")


def plummer_positions(rng, count, a, r_trunc):
    """Textbook Plummer sphere radii r = a / sqrt(u^(-2/3) - 1), truncated."""
    out = np.empty((0, 3))
    while out.shape[0] < count:
        k = count - out.shape[0]
        u = rng.uniform(1e-12, 1.0, k)
        rad = a / np.sqrt(u ** (-2.0 / 3.0) - 1.0)
        xi = rng.uniform(-1.0, 1.0, k)
        zeta = rng.uniform(0.0, 2.0 * np.pi, k)
        st = np.sqrt(1.0 - xi * xi)
        x = np.stack([st * np.cos(zeta), st * np.sin(zeta), xi], axis=1) * rad[:, None]
        out = np.concatenate([out, x[rad <= r_trunc]], axis=0)
    return out[:count]


def plummer_mixture(seed=0, N=1 << 24, n=512, clumps=8, a_range=(8.0, 32.0),
                    log_mass_decades=1.0, M=1.0, G=1.0, a0=None):
    """Mixture of Plummer spheres (a build choice; the paper has no Plummer model).

    Radii a_j ~ U[a_range] cells, masses log-uniform over the given number of
    decades, normalised to M; particles proportional to mass; centres uniform
    but kept 5 a_j + 4 cells inside the physical region; per-clump Maxwellian
    <v^2> = (2/3) sqrt(G m_j a0).  If a0 is None it is G M / (2 r_h^2) with
    r_h the half-mass radius about the centre of mass.
    """
    rng = np.random.default_rng(seed)
    a = rng.uniform(a_range[0], a_range[1], clumps)
    lm = rng.uniform(0.0, log_mass_decades, clumps)
    mj = 10.0 ** lm
    mj = M * mj / mj.sum()
    counts = np.floor(mj / M * N).astype(np.int64)
    counts[np.argmax(counts)] += N - counts.sum()
    half = n / 2.0
    pos_l = []
    for j in range(clumps):
        lim = max(half - (5.0 * a[j] + 4.0), 0.0)
        c = rng.uniform(-lim, lim, 3)
        pos_l.append(plummer_positions(rng, int(counts[j]), a[j], 5.0 * a[j]) + c)
    pos = np.concatenate(pos_l, axis=0)
    mass = np.full(N, M / N)
    com = pos.mean(axis=0)
    if a0 is None:
        r_h = float(np.median(np.linalg.norm(pos - com, axis=1)))
        a0 = G * M / (2.0 * r_h * r_h)
    vel = np.concatenate([maxwellian(rng, int(counts[j]),
                                     2.0 / 3.0 * math.sqrt(G * mj[j] * a0))
                          for j in range(clumps)], axis=0)
    p = params(n, a0=a0, mu=MU_STANDARD, sigma=1.0, G=G)
    pos, vel, mass = _f32(pos, vel, mass)
    return dict(params=p, pos=pos, vel=vel, mass=mass, dt=0.5, steps=10,
                workload=f"plummer_mix_{n}_N{N}")


def random_cloud(seed, n, N, radius_frac=0.35, mass_range=(0.5, 1.5), mu=MU_STANDARD,
                 a0=None, sigma=1.0, G=1.0, iters=4, n_pad=None, vmax=0.1):
    """Uniform random particles in a ball in the central physical region.

    A generic parity workload: masses uniform in mass_range, positions uniform
    in a ball of radius radius_frac * n cells, velocities uniform in
    [-vmax, vmax].  a0 defaults to the Newtonian field of the total mass at
    the ball radius, so that both regimes of the interpolation occur.
    """
    rng = np.random.default_rng(seed)
    R = radius_frac * n
    u = rng.standard_normal((N, 3))
    u /= np.linalg.norm(u, axis=1, keepdims=True)
    rad = R * rng.uniform(0.0, 1.0, N) ** (1.0 / 3.0)
    pos = u * rad[:, None]
    vel = rng.uniform(-vmax, vmax, (N, 3))
    mass = rng.uniform(mass_range[0], mass_range[1], N)
    if a0 is None:
        a0 = G * float(mass.sum()) / (R * R)
    p = params(n, n_pad=n_pad, a0=a0, mu=mu, sigma=sigma, G=G, iters=iters)
    pos, vel, mass = _f32(pos, vel, mass)
    return dict(params=p, pos=pos, vel=vel, mass=mass, dt=0.1,
                workload=f"cloud_{n}_N{N}")


def lone_particle(seed, n=64, count=1, mu=MU_DEEP, a0=1e3, sigma=1.0):
    """One particle at random sub-pixel offsets near the origin (self-force)."""
    rng = np.random.default_rng(seed)
    offs = rng.uniform(-0.5, 0.5, (count, 3))
    p = params(n, a0=a0, mu=mu, sigma=sigma)
    return dict(params=p, offsets=offs.astype(np.float32), mass=np.ones(1, np.float32))


def mixture_training_sample(seed, n=128, N_range=(16, 18), clumps_range=(2, 16),
                            a_range=(2.0, 8.0), M=1.0, G=1.0, a0=None):
    """Random Plummer mixture used as a training input for the learned start.

    Clumps ~ U{clumps_range}, N = round(2^u) with u ~ U[N_range], radii
    log-uniform over a_range (cells), centres kept 5a+4 cells inside the
    physical region.  Standard interpolation; a0 as in plummer_mixture.
    """
    rng = np.random.default_rng(seed)
    clumps = int(rng.integers(clumps_range[0], clumps_range[1] + 1))
    N = int(round(2.0 ** rng.uniform(N_range[0], N_range[1])))
    a = np.exp(rng.uniform(math.log(a_range[0]), math.log(a_range[1]), clumps))
    mj = 10.0 ** rng.uniform(0.0, 1.0, clumps)
    mj = M * mj / mj.sum()
    counts = np.maximum(np.floor(mj / M * N).astype(np.int64), 1)
    counts[np.argmax(counts)] += N - counts.sum()
    half = n / 2.0
    pos_l = []
    for j in range(clumps):
        lim = max(half - (5.0 * a[j] + 4.0), 0.0)
        c = rng.uniform(-lim, lim, 3)
        pos_l.append(plummer_positions(rng, int(counts[j]), a[j], 5.0 * a[j]) + c)
    pos = np.concatenate(pos_l, axis=0)
    mass = np.full(pos.shape[0], M / pos.shape[0])
    if a0 is None:
        com = pos.mean(axis=0)
        r_h = float(np.median(np.linalg.norm(pos - com, axis=1)))
        a0 = G * M / (2.0 * r_h * r_h)
    p = params(n, a0=a0, mu=MU_STANDARD, sigma=1.0, G=G)
    pos, mass = _f32(pos, mass)
    return dict(params=p, pos=pos, mass=mass, workload=f"mixture_{n}_s{seed}")
