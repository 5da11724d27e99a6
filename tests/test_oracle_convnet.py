"""Pins of the learned-start oracle (network, its gradients, Adam, the input
features and the start field).  The network is not in the paper, so these
pins come from definitions: brute-force sums, adjoint identities, finite
differences of the loss, the closed form of Adam's first step and a library
BF16 conversion."""
import math

import numpy as np
import pytest
import torch

from oracle import convnet as cn
from oracle import learned as ol
from oracle import pm


def test_conv3d_brute_force():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((2, 4, 3, 5))
    w = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(3)
    got = cn.conv3d(x, w, b)
    C, D, H, W = x.shape
    for o in range(3):
        for z in range(D):
            for y in range(H):
                for xx in range(W):
                    s = b[o]
                    t = 0
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                zz, yy, x2 = z + dz, y + dy, xx + dx
                                if 0 <= zz < D and 0 <= yy < H and 0 <= x2 < W:
                                    for c in range(C):
                                        s += x[c, zz, yy, x2] * w[t, c, o]
                                t += 1
                    assert abs(got[o, z, y, xx] - s) < 1e-12


def test_periodic_conv3d_brute_force():
    rng = np.random.default_rng(10)
    x = rng.standard_normal((2, 4, 3, 5))
    w = rng.standard_normal((27, 2, 3))
    b = rng.standard_normal(3)
    got = cn.conv3d(x, w, b, periodic=True)
    C, D, H, W = x.shape
    for o in range(3):
        for z in range(D):
            for y in range(H):
                for xx in range(W):
                    s = b[o]
                    t = 0
                    for dz in (-1, 0, 1):
                        for dy in (-1, 0, 1):
                            for dx in (-1, 0, 1):
                                for c in range(C):
                                    s += x[c, (z + dz) % D, (y + dy) % H, (xx + dx) % W] * w[t, c, o]
                                t += 1
                    assert abs(got[o, z, y, xx] - s) < 1e-12


def test_conv3d_delta_response_fixes_tap_orientation():
    # a unit impulse at v0 in channel c gives out[o, v0 - tap_t] = w[t, c, o]
    rng = np.random.default_rng(1)
    w = rng.standard_normal((27, 3, 2))
    x = np.zeros((3, 5, 5, 5))
    x[1, 2, 2, 2] = 1.0
    out = cn.conv3d(x, w, np.zeros(2))
    t = 0
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                assert np.allclose(out[:, 2 - dz, 2 - dy, 2 - dx], w[t, 1])
                t += 1


@pytest.mark.parametrize("taps,periodic", [(27, False), (1, False), (27, True)])
def test_conv_backward_is_the_adjoint(taps, periodic):
    rng = np.random.default_rng(2)
    x = rng.standard_normal((3, 4, 4, 6))
    w = rng.standard_normal((taps, 3, 5))
    g = rng.standard_normal((5, 4, 4, 6))
    y = cn.conv3d(x, w, np.zeros(5), periodic)
    gx, gw, gb = cn.conv3d_backward(x, w, g, periodic)
    ip = float((y * g).sum())
    assert abs(ip - float((gx * x).sum())) < 1e-10 * abs(ip)
    assert abs(ip - float((gw * w).sum())) < 1e-10 * abs(ip)
    assert np.allclose(gb, g.sum(axis=(1, 2, 3)))


def test_pool_and_upsample_adjoints():
    rng = np.random.default_rng(3)
    a = rng.standard_normal((2, 4, 6, 8))
    b = rng.standard_normal((2, 2, 3, 4))
    assert abs(float((cn.pool2(a) * b).sum()) - float((a * cn.pool2_backward(b)).sum())) < 1e-12
    assert abs(float((cn.up2(b) * a).sum()) - float((b * cn.up2_backward(a)).sum())) < 1e-12
    assert np.allclose(cn.pool2(cn.up2(b)), b)
    assert cn.pool2(a)[1, 0, 1, 2] == pytest.approx(a[1, 0:2, 2:4, 4:6].mean())


def test_parameter_count():
    p = cn.init_params(0)
    n = sum(v.size for v in p.values())
    assert n == sum(k ** 3 * ci * co + co for _, ci, co, k in cn.LAYERS)
    assert 3.0e5 < n < 4.0e5


def _loss(p, x, t, periodic=False):
    y, _ = cn.forward(p, x, periodic=periodic)
    return cn.mse(y, t)[0]


@pytest.mark.parametrize("periodic", [False, True])
def test_network_gradient_matches_finite_differences(periodic):
    rng = np.random.default_rng(4)
    p = cn.init_params(1)
    for k in p:
        if k.endswith(".b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    x = rng.standard_normal((4, 8, 8, 8))
    t = rng.standard_normal((3, 8, 8, 8))
    y, cache = cn.forward(p, x, periodic=periodic)
    _, gy = cn.mse(y, t)
    g = cn.backward(p, cache, gy)
    eps = 1e-6
    for k in p:
        flat = p[k].reshape(-1)
        for i in rng.choice(flat.size, size=min(3, flat.size), replace=False):
            old = flat[i]
            flat[i] = old + eps
            lp = _loss(p, x, t, periodic)
            flat[i] = old - eps
            lm = _loss(p, x, t, periodic)
            flat[i] = old
            fd = (lp - lm) / (2 * eps)
            an = g[k].reshape(-1)[i]
            # FD rounding: about 1e-16 loss / eps = 1e-10
            assert abs(fd - an) <= 1e-5 * abs(an) + 1e-9, (k, i, fd, an)


def test_bf16_rounding_matches_torch():
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(5000) * 10.0 ** rng.integers(-30, 30, 5000),
                        1.0 + np.array([1, 2, 3, 5]) * 2.0 ** -8,      # ties and near-ties
                        [-(1.0 + 3 * 2.0 ** -8), 0.0, -0.0]]).astype(np.float32)
    ref = torch.from_numpy(v).to(torch.bfloat16).float().numpy().astype(np.float64)
    assert np.array_equal(cn.bf16_round(v), ref)
    assert cn.bf16_round(np.float32(1 + 2 ** -8)) == 1.0                 # tie to even
    assert cn.bf16_round(np.float32(1 + 3 * 2 ** -8)) == 1 + 2 ** -6


def test_adam_first_step_closed_form():
    # after one step with zero moments, m_hat = g and v_hat = g^2, so each
    # parameter moves by lr g / (|g| + eps)
    rng = np.random.default_rng(6)
    p = {"a": rng.standard_normal(10)}
    g = {"a": rng.standard_normal(10)}
    p0 = p["a"].copy()
    st = {}
    cn.adam_step(p, g, st, lr=0.01)
    assert np.allclose(p["a"], p0 - 0.01 * g["a"] / (np.abs(g["a"]) + 1e-8), rtol=1e-12)
    # a constant gradient keeps the step at lr
    for _ in range(5):
        cn.adam_step(p, {"a": np.full(10, 0.3)}, st, lr=0.01)
    q = {"a": p["a"].copy()}
    st2 = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in st.items()}
    cn.adam_step(q, {"a": np.full(10, 0.3)}, st2, lr=0.01)
    assert np.all(q["a"] < p["a"])


def test_training_reduces_loss_on_a_fixed_pair():
    rng = np.random.default_rng(7)
    p = cn.init_params(2, scale=0.5)
    x = rng.standard_normal((4, 8, 8, 8))
    t = 0.3 * x[:3] + 0.1
    st = {}
    l0 = _loss(p, x, t)
    for _ in range(30):
        y, cache = cn.forward(p, x)
        _, gy = cn.mse(y, t)
        cn.adam_step(p, cn.backward(p, cache, gy), st, lr=1e-3)
    assert _loss(p, x, t) < 0.5 * l0


def test_net_input_and_start_field():
    # the network sees the whole box averaged over 2 x 2 x 2 blocks
    p = pm.Params(n=8, n_pad=16, box=8.0, a0=2.0)
    rng = np.random.default_rng(8)
    gN = rng.standard_normal((3, 16, 16, 16))
    x, rms = ol.net_input(p, gN)
    assert x.shape == (4, 8, 8, 8)
    gc = np.zeros((3, 8, 8, 8))
    for dz in (0, 1):
        for dy in (0, 1):
            for dx in (0, 1):
                gc += gN[:, dz::2, dy::2, dx::2] / 8.0
    assert rms == pytest.approx(math.sqrt((gc ** 2).sum() / 8 ** 3))
    assert np.allclose(x[:3], gc / rms)
    assert np.allclose(10.0 ** x[3], np.sqrt((gc ** 2).sum(axis=0)) / 2.0 + 1e-30)
    y = rng.standard_normal((3, 8, 8, 8))
    H0 = ol.start_field(p, y, rms)
    assert H0.shape == (3, 16, 16, 16)
    assert np.allclose(H0[:, 5, 9, 14], rms * y[:, 2, 4, 7])
    assert np.allclose(ol.target(p, H0, rms), y)


def test_net_input_and_start_field_at_quarter_resolution():
    # f = 4: the network sees the box averaged over 4 x 4 x 4 blocks
    p = pm.Params(n=8, n_pad=16, box=8.0, a0=2.0)
    rng = np.random.default_rng(9)
    gN = rng.standard_normal((3, 16, 16, 16))
    x, rms = ol.net_input(p, gN, f=4)
    assert x.shape == (4, 4, 4, 4)
    gc = np.zeros((3, 4, 4, 4))
    for Z in range(4):
        for Y in range(4):
            for X in range(4):
                gc[:, Z, Y, X] = gN[:, 4 * Z:4 * Z + 4, 4 * Y:4 * Y + 4, 4 * X:4 * X + 4].sum(axis=(1, 2, 3)) / 64.0
    assert rms == pytest.approx(math.sqrt((gc ** 2).sum() / 4 ** 3))
    assert np.allclose(x[:3], gc / rms)
    y = rng.standard_normal((3, 4, 4, 4))
    H0 = ol.start_field(p, y, rms, f=4)
    assert H0.shape == (3, 16, 16, 16)
    assert np.allclose(H0[:, 5, 9, 14], rms * y[:, 1, 2, 3])
    assert np.allclose(ol.target(p, H0, rms, f=4), y)


@pytest.mark.parametrize("f", [2, 4])
def test_start_field_spectrum_is_coarse_spectrum_times_block_sums(f):
    # The learned solve never forms the full-resolution start: it multiplies
    # the coarse output's n^3-point DFT by the DFT of one block of f cells
    # per axis.  For the start the oracle builds (each coarse value repeated
    # over its f^3 block), DFT_N(H0)(k) = Y(k mod n) B(kx) B(ky) B(kz) with
    # Y = DFT_n(rms y) and B(k) = sum_{j < f} exp(-2 pi i k j / N).
    n = 4
    N = f * n
    rng = np.random.default_rng(21)
    y = rng.standard_normal((3, n, n, n))
    H0 = ol.start_field(None, y, 1.7, f)
    assert H0.shape == (3, N, N, N)
    Y = np.fft.fftn(1.7 * y, axes=(1, 2, 3))
    k = np.arange(N)
    B = np.exp(-2j * np.pi * np.outer(k, np.arange(f)) / N).sum(axis=1)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    want = Y[:, kz % n, ky % n, kx % n] * (B[kz] * B[ky] * B[kx])[None]
    got = np.fft.fftn(H0, axes=(1, 2, 3))
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(got))


@pytest.mark.parametrize("f", [2, 4])
def test_feature_block_means_are_aliases_of_the_newton_spectrum(f):
    # The learned solve forms the network's block means of g_N = -D phi_N
    # without a real phi_N: their n^3-point DFT is
    # (1/f^3) sum_{k = K mod n} -i kappa(k) phi_hat(k) conj(B(kx) B(ky) B(kz)),
    # kappa the central-difference symbol sin(2 pi k / N) / s, phi_hat the
    # normalised spectrum (phi = sum phi_hat e^{+ikx}) and B as for the start.
    # Checked on the oracle's own Newton potential and block means.
    p = pm.Params(n=8, n_pad=16, box=5.0)
    N, n = p.n_pad, p.n_pad // f
    rng = np.random.default_rng(31)
    rho = np.zeros((N, N, N))
    rho[4:12, 4:12, 4:12] = rng.uniform(0.0, 1.0, (8, 8, 8))
    phiN, gN = pm.newton_potential(p, rho)
    want = ol.coarse(gN, f)
    ph = np.fft.fftn(phiN) / N ** 3
    k = np.arange(N)
    kap = np.sin(2 * np.pi * k / N) / p.s
    B = np.exp(-2j * np.pi * np.outer(k, np.arange(f)) / N).sum(axis=1)
    kz, ky, kx = np.meshgrid(k, k, k, indexing="ij")
    w = ph * np.conj(B[kz] * B[ky] * B[kx]) / f ** 3
    Y = np.zeros((3, n, n, n), complex)
    for c, kc in enumerate((kx, ky, kz)):
        np.add.at(Y[c], (kz % n, ky % n, kx % n), -1j * kap[kc] * w)
    got = np.fft.ifftn(Y, axes=(1, 2, 3)).real * n ** 3
    assert np.max(np.abs(got - want)) < 1e-12 * np.max(np.abs(want))
