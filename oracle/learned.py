"""FP64 oracle of the learned starting guess around the network (test
infrastructure: only tests, the smoke check and the benchmark's CPU baseline
leg may use this module).

The fixed-point iteration of Sect. 2.1 may start from any divergence-free H;
the paper starts from zero and notes that a good start (its example: the H of
the previous time step) cuts the iterations needed.  Here the start is
predicted from the Newton field (parity unpinned against the paper, which has
no network).  H lives on the whole periodic n_pad^3 box, half of it outside
the physical region, so the network sees the whole box at half (f = 2) or
quarter (f = 4) resolution:

    g_c   = mean of g_N over each f x f x f block of the box ((n_pad/f)^3)
    rms   = sqrt(mean of |g_c|^2)
    x     = [g_c / rms (3 channels), log10(|g_c| / a0 + 1e-30)]
    y_hat = net(x), periodic convolutions       (3 channels, (n_pad/f)^3)
    H0    = rms * y_hat, each value repeated over its f x f x f block

and the solver takes the divergence-free part of H0.  The training target for
a solved field H* is the block mean of H* divided by rms.
"""
from __future__ import annotations

import math

import numpy as np

from . import pm


def coarse(a, f=2):
    """Mean over f x f x f blocks of the last three axes."""
    C, D, H, W = a.shape
    return a.reshape(C, D // f, f, H // f, f, W // f, f).mean(axis=(2, 4, 6))


def fine(a, f=2):
    """Each value repeated over an f x f x f block (inverse of coarse on such fields)."""
    return np.repeat(np.repeat(np.repeat(a, f, axis=1), f, axis=2), f, axis=3)


def newton_field(p: pm.Params, rho):
    """g_N on the whole box (flow scheme: Newton potential, then the
    finite-difference gradient)."""
    _, gN = pm.newton_potential(p, rho)
    return gN


def net_input(p: pm.Params, gN, f=2):
    """Network input [4, n_pad/f, n_pad/f, n_pad/f] and the scale rms."""
    g = coarse(gN, f)
    mag = np.sqrt((g * g).sum(axis=0))
    rms = math.sqrt(float((mag * mag).mean()))
    scale = 1.0 / rms if rms > 0.0 else 0.0
    x = np.concatenate([g * scale, np.log10(mag / p.a0 + 1e-30)[None]], axis=0)
    return x, rms


def start_field(p: pm.Params, y_hat, rms, f=2):
    """H0 [3, n_pad, n_pad, n_pad] = rms * y_hat repeated over f x f x f blocks."""
    return rms * fine(np.asarray(y_hat, dtype=np.float64), f)


def target(p: pm.Params, H, rms, f=2):
    """Training target: block mean of the solved H divided by rms."""
    return coarse(H, f) / rms
