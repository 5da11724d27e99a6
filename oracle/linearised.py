"""FP64 oracle of the linearised incremental field update (Sect. 5, item (v)).

TEST INFRASTRUCTURE: only tests, the smoke check and the benchmark's CPU
baseline leg may use this module (see the package docstring).

The paper proposes to carry the step-to-step increments of the fields
instead of the fields when they change little between steps, with the two
algebraic equations (Eqs. inverse and interpolation) replaced by their
linearisations about the previous fields:

    dg_M = nu(F/a0) dF + nu'(F/a0) (F . dF) / (a0 F) F
    dF   = mu(g_M/a0) dg_M + mu'(g_M/a0) (g_M . dg_M) / (a0 g_M) g_M

while the linear parts (Eq. newtongrav for dg_N, the curl-free and the
divergence-free projections) act on increments unchanged.  The increments
are small, so they can be stored with few significant digits (half
precision, Sect. 5, item (iv)).

``incremental_solve`` runs the fixed-point iteration of Sect. 2.1 on the
increments in the same order as ``pm.aqual_solve`` runs it on the fields:
dF = dg_N + dH; dg_M from the first linearisation; project curl-free
(giving dphi); dF' from the second linearisation; dH = the divergence-free
part of dF' - dg_N.  ``store`` rounds every stored increment field; the
transforms themselves stay FP64.

Reading (the paper gives only the two formulas): half-precision storage is
modelled as FP16 rounding of each increment field after division by one
power-of-two scale per field (the smallest power of two not below its
largest magnitude), so that small increments are not lost to FP16's range.
"""
from __future__ import annotations

import math

import numpy as np

from . import pm

__all__ = ["nu_value", "nu_slope", "mu_value", "mu_slope", "linearised_nu",
           "linearised_mu", "to_half", "base_state", "incremental_solve", "advance_base"]


def nu_value(p: pm.Params, y: np.ndarray) -> np.ndarray:
    """nu(y) for y = |F|/a0 > 0: the inverse of the chosen mu (Eq. mu and the nu
    printed after it).  Standard: nu^2 = 1/2 + sqrt(1/4 + 1/y^2); deep MOND:
    nu = y^(-1/2); Newton: nu = 1."""
    if p.mu == pm.MU_NEWTON:
        return np.ones_like(y)
    if p.mu == pm.MU_DEEP:
        return 1.0 / np.sqrt(y)
    return np.sqrt(0.5 + np.sqrt(0.25 + 1.0 / (y * y)))


def nu_slope(p: pm.Params, y: np.ndarray) -> np.ndarray:
    """nu'(y), from differentiating nu_value: standard 2 nu nu' = -(1/y^3) /
    sqrt(1/4 + 1/y^2); deep MOND -y^(-3/2)/2; Newton 0."""
    if p.mu == pm.MU_NEWTON:
        return np.zeros_like(y)
    if p.mu == pm.MU_DEEP:
        return -0.5 * y ** -1.5
    return -1.0 / (2.0 * nu_value(p, y) * y ** 3 * np.sqrt(0.25 + 1.0 / (y * y)))


def mu_value(p: pm.Params, x: np.ndarray) -> np.ndarray:
    """mu(x): standard x / sqrt(1 + x^2) (Eq. mu); deep MOND x; Newton 1."""
    if p.mu == pm.MU_NEWTON:
        return np.ones_like(x)
    if p.mu == pm.MU_DEEP:
        return x.copy()
    return x / np.sqrt(1.0 + x * x)


def mu_slope(p: pm.Params, x: np.ndarray) -> np.ndarray:
    """mu'(x): standard (1 + x^2)^(-3/2); deep MOND 1; Newton 0."""
    if p.mu == pm.MU_NEWTON:
        return np.zeros_like(x)
    if p.mu == pm.MU_DEEP:
        return np.ones_like(x)
    return (1.0 + x * x) ** -1.5


def _linearised(value, slope, p: pm.Params, A: np.ndarray, dA: np.ndarray) -> np.ndarray:
    """f(|A|/a0) dA + f'(|A|/a0) (A . dA) / (a0 |A|) A, zero where A = 0 (the
    map A -> f(|A|/a0) A has no derivative there for MOND's f)."""
    Am = np.sqrt((A * A).sum(axis=0))
    nz = Am > 0.0
    safe = np.where(nz, Am, 1.0)
    t = safe / p.a0
    f = value(p, t)
    fp = slope(p, t)
    dot = (A * dA).sum(axis=0)
    out = f * dA + (fp * dot / (p.a0 * safe)) * A
    return np.where(nz, out, 0.0)


def linearised_nu(p: pm.Params, F: np.ndarray, dF: np.ndarray) -> np.ndarray:
    """dg_M from dF, linearised about F (Sect. 5, item (v), first formula)."""
    return _linearised(nu_value, nu_slope, p, F, dF)


def linearised_mu(p: pm.Params, gM: np.ndarray, dgM: np.ndarray) -> np.ndarray:
    """dF from dg_M, linearised about g_M (Sect. 5, item (v), second formula)."""
    return _linearised(mu_value, mu_slope, p, gM, dgM)


def to_half(a: np.ndarray) -> np.ndarray:
    """FP16 storage of one increment field with a power-of-two scale (the
    reading in the module docstring); returned as FP64."""
    m = float(np.abs(a).max()) if a.size else 0.0
    if m == 0.0:
        return np.zeros_like(a)
    scale = 2.0 ** math.ceil(math.log2(m))
    return (a / scale).astype(np.float16).astype(np.float64) * scale


def base_state(p: pm.Params, rho: np.ndarray, tol: float = 1e-13, max_iters: int = 200):
    """The fields of the previous step, solved to convergence: g_N, H, F = g_N + H,
    g_M = the curl-free part of nu(F) F, and phi (Sect. 2.1)."""
    q = pm.Params(**{**p.__dict__, "iters": max_iters, "tol": tol})
    phi, info = pm.aqual_solve(q, rho, keep_fields=True)
    F = info.gN + info.H
    gh, _ = pm.project_curl_free(q, np.stack([pm.fft3(c) for c in pm.apply_nu(q, F)]))
    gM = np.stack([pm.ifft3_real(c) for c in gh])
    return dict(gN=info.gN, H=info.H, F=F, gM=gM, phi=phi, info=info)


def incremental_solve(p: pm.Params, base: dict, d_rho: np.ndarray, iters: int,
                      store=None, keep_fields: bool = False):
    """dphi for a density increment d_rho about ``base`` (Sect. 5, item (v)),
    with ``iters`` evaluations of the first linearisation from dH = 0.

    Returns (dphi, residuals), residuals r_k = ||dH_k - dH_{k-1}|| / ||dg_N||.
    ``store`` (identity by default) is applied to dg_N, dF, dg_M and dH where
    they would be written to memory.  With keep_fields the increments of the
    last iteration are returned as a third item: dg_N, dH, dF = dg_N + dH and
    dg_M (the curl-free part of the last linearised nu), as ``advance_base``
    takes them.
    """
    if store is None:
        def store(a):
            return a
    _, dgN = pm.newton_potential(p, d_rho)
    dgN = store(dgN)
    norm = math.sqrt(float((dgN * dgN).sum()))
    dH = np.zeros_like(dgN)
    res = []
    dphih = None
    dF = dgM = None
    K = max(int(iters), 1)
    for k in range(1, K + 1):
        dF = store(dgN + dH)
        dgM = linearised_nu(p, base["F"], dF)
        gh, dphih = pm.project_curl_free(p, np.stack([pm.fft3(c) for c in dgM]))
        if k == K:
            if keep_fields:
                dgM = store(np.stack([pm.ifft3_real(c) for c in gh]))
            break
        dgM = store(np.stack([pm.ifft3_real(c) for c in gh]))
        dFp = linearised_mu(p, base["gM"], dgM)
        Hh = pm.project_div_free(p, np.stack([pm.fft3(c) for c in dFp - dgN]))
        dHn = store(np.stack([pm.ifft3_real(c) for c in Hh]))
        d = dHn - dH
        res.append(math.sqrt(float((d * d).sum())) / norm if norm > 0 else 0.0)
        dH = dHn
    dphi = pm.ifft3_real(dphih)
    if keep_fields:
        return dphi, res, dict(dgN=dgN, dH=dH, dF=dF, dgM=dgM)
    return dphi, res


def advance_base(base: dict, dphi: np.ndarray, inc: dict) -> dict:
    """The next step's previous fields: every field plus its increment, so that
    the next increment is linearised about the updated F and g_M."""
    return dict(gN=base["gN"] + inc["dgN"], H=base["H"] + inc["dH"], F=base["F"] + inc["dF"],
                gM=base["gM"] + inc["dgM"], phi=base["phi"] + dphi, info=base.get("info"))
