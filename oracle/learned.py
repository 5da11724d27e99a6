"""FP64 oracle of the learned starting guess around the network (test
infrastructure: only tests, the smoke check and the benchmark's CPU baseline
leg may use this module).

The fixed-point iteration of Sect. 2.1 may start from any divergence-free H;
the paper starts from zero and notes that a good start (its example: the H of
the previous time step) cuts the iterations needed.  Here the start is
predicted from the Newton field on the physical n^3 region (parity unpinned
against the paper, which has no network):

    rms   = sqrt(mean over the region of |g_N|^2)
    x     = [g_N / rms (3 channels), log10(|g_N| / a0 + 1e-30)]
    y_hat = net(x)                           (3 channels, the region)
    H0    = zero extension of rms * y_hat to the n_pad^3 box

and the solver takes the divergence-free part of H0.  The training target
for a solved field H* is H* / rms on the region.
"""
from __future__ import annotations

import math

import numpy as np

from . import pm


def region(p: pm.Params):
    """Index slice of the physical n^3 region inside the n_pad^3 box (the
    n cells centred on the box centre, Sect. 3)."""
    lo = p.n_pad // 2 - p.n // 2
    return slice(lo, lo + p.n)


def newton_field(p: pm.Params, rho):
    """g_N on the whole box (flow scheme: Newton potential, then the
    finite-difference gradient)."""
    _, gN = pm.newton_potential(p, rho)
    return gN


def net_input(p: pm.Params, gN):
    """Network input [4, n, n, n] and the scale rms."""
    r = region(p)
    g = gN[:, r, r, r]
    mag = np.sqrt((g * g).sum(axis=0))
    rms = math.sqrt(float((mag * mag).mean()))
    scale = 1.0 / rms if rms > 0.0 else 0.0
    x = np.concatenate([g * scale, np.log10(mag / p.a0 + 1e-30)[None]], axis=0)
    return x, rms


def start_field(p: pm.Params, y_hat, rms):
    """H0 [3, n_pad, n_pad, n_pad]: rms * y_hat on the region, zero outside."""
    r = region(p)
    H0 = np.zeros((3, p.n_pad, p.n_pad, p.n_pad))
    H0[:, r, r, r] = rms * np.asarray(y_hat, dtype=np.float64)
    return H0


def target(p: pm.Params, H, rms):
    """Training target: the solved H on the region divided by rms."""
    r = region(p)
    return H[:, r, r, r] / rms
