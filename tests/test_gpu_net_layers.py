"""Per-layer parity of the learned start's kernels with the FP64 oracle.

Each oracle layer is fed the GPU's own stored BF16 input for that layer (read
back with pm_net_get_tensor) and the same BF16 weights.  Where the GPU stores
a BF16 result, the check is that every stored value is one of the two BF16
numbers around the exact FP64 result (FP32 accumulation may pick the other
neighbour when the exact value lies close to a rounding midpoint), and that
the relative L2 distance to the exact result rounded to BF16 stays below
2e-4 (a handful of such one-step flips; measured 1e-5 to 1.3e-4 on 32- and
64-channel layers, whose sums run over 864 and 1728 terms).  FP32 results
(the head, weight and bias gradients) are checked at 1e-4 relative L2.
Covered: every convolution, pooling and upsampling (forward), the head,
every backward-data convolution and gradient combination whose inputs the
GPU still holds after a backward pass, and every weight and bias gradient.
The gradients of the four decoder layers need upstream gradients the GPU
overwrites later in the pass; the oracle rebuilds those from the head with
the same BF16 roundings."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import convnet as cn  # noqa: E402
from tests.gpu_util import dev, host, rel_l2  # noqa: E402
from tests.test_gpu_net import M, gpu_params, net_inputs, unflat  # noqa: E402

BAR = 1e-4          # FP32 results
BAR_BF16 = 2e-4     # BF16 results, against the exact value rounded to BF16
r = cn.bf16_round


def bf16_step(x):
    """Spacing of the BF16 numbers at |x| (8 significant bits)."""
    ax = np.abs(x)
    e = np.floor(np.log2(np.where(ax > 0, ax, 1.0)))
    return np.where(ax > 0, 2.0 ** (e - 7), 0.0)


def conv(a, p, name, periodic=True):
    return cn.conv3d(a, p[name + ".w"], p[name + ".b"], periodic)


def convT(g, p, name):
    """Gradient of a (periodic) convolution with respect to its input."""
    w = p[name + ".w"]
    x0 = np.zeros((w.shape[1],) + g.shape[1:])
    ga, _, _ = cn.conv3d_backward(x0, w, g, True)
    return ga


def wgrad(a, g, p, name):
    _, gw, gb = cn.conv3d_backward(a, p[name + ".w"], g, True)
    return gw, gb


@pytest.mark.parametrize("n,batch", [(16, 2), (64, 1)])
def test_net_layers_match_oracle(n, batch):
    rng = np.random.default_rng(31 + n)
    v32, po = gpu_params(5)
    net = M.Net(n, batch)
    M.pm_net_set_params(net, v32)
    ts = []
    for b in range(batch):
        M.pm_net_set_input(net, b, dev(net_inputs(rng, n)))
        t = (0.5 * rng.standard_normal((3, n, n, n))).astype(np.float32)
        M.pm_net_set_target(net, b, dev(t))
        ts.append(t.astype(np.float64))
    M.pm_net_backward(net, batch)
    gpu_g = unflat(M.pm_net_get_grads(net).astype(np.float64))
    ora_g = {k: np.zeros_like(v) for k, v in po.items()}
    worst = {}

    def check(name, got, ref, bar=BAR):
        e = rel_l2(got, ref)
        worst[name] = max(worst.get(name, 0.0), e)
        assert e < bar, (name, e)

    def check16(name, got, exact, strict=True):
        """got: stored BF16 values; exact: the FP64 result before rounding
        (strict: from exactly the GPU's inputs, so every value must be one of
        its two BF16 neighbours)."""
        floor = 2.0 ** -20 * np.abs(exact).max()          # FP32 accumulation of cancelling terms
        if strict:
            assert np.all(np.abs(got - exact) <= bf16_step(exact) + floor), name
        check(name, got, r(exact), BAR_BF16)

    for b in range(batch):
        T = {k: host(M.pm_net_get_tensor(net, k, b)) for k in M.NET_TENSORS}
        yhat = host(M.pm_net_output(net, b, torch.empty(3 * n ** 3, device="cuda"))).reshape(3, n, n, n)
        relu = lambda z: np.maximum(z, 0.0)  # noqa: E731
        cat2 = np.concatenate([T["s2"], cn.up2(T["b3"])])
        cat1 = np.concatenate([T["s1"], cn.up2(T["d2"])])
        # forward, one layer at a time from the GPU's stored inputs
        check16("e1a", T["a1"], relu(conv(T["x"], po, "e1a")))
        check16("e1b", T["s1"], relu(conv(T["a1"], po, "e1b")))
        check16("pool1", T["p1"], cn.pool2(T["s1"]))
        check16("e2a", T["a2"], relu(conv(T["p1"], po, "e2a")))
        check16("e2b", T["s2"], relu(conv(T["a2"], po, "e2b")))
        check16("pool2", T["p2"], cn.pool2(T["s2"]))
        check16("b3a", T["a3"], relu(conv(T["p2"], po, "b3a")))
        check16("b3b", T["b3"], relu(conv(T["a3"], po, "b3b")))
        check16("d2a (skip + upsampled)", T["a4"], relu(conv(cat2, po, "d2a")))
        check16("d2b", T["d2"], relu(conv(T["a4"], po, "d2b")))
        check16("d1a (skip + upsampled)", T["a5"], relu(conv(cat1, po, "d1a")))
        check16("d1b", T["d1"], relu(conv(T["a5"], po, "d1b")))
        check("head", yhat, conv(T["d1"], po, "out"), 1e-6)
        # backward: the loss is the mean over slots, channels and voxels; the
        # GPU forms dL/dy in FP32 and rounds every stored gradient to BF16
        count = 3.0 * n ** 3 * batch
        gy = (2.0 * (yhat - ts[b]) / count).astype(np.float32).astype(np.float64)
        gz_d1b = r((T["d1"] > 0) * convT(gy, po, "out"))
        gz_d1a = r((T["a5"] > 0) * convT(gz_d1b, po, "d1b"))
        check16("gc1 = d1a backward data", T["gc1"], convT(gz_d1a, po, "d1a"), strict=False)
        gz_d2b = r((T["d2"] > 0) * cn.up2_backward(T["gc1"][16:]))
        gz_d2a = r((T["a4"] > 0) * convT(gz_d2b, po, "d2b"))
        check16("gc2 = d2a backward data", T["gc2"], convT(gz_d2a, po, "d2a"), strict=False)
        check16("b3b upsampling gradient", T["g64a"], (T["b3"] > 0) * cn.up2_backward(T["gc2"][32:]))
        check16("b3b backward data", T["g64b"], (T["a3"] > 0) * convT(T["g64a"], po, "b3b"))
        check16("b3a backward data", T["gp2"], convT(T["g64b"], po, "b3a"))
        check16("level 2 pooling gradient", T["g32a"],
                (T["s2"] > 0) * (T["gc2"][:32] + cn.pool2_backward(T["gp2"])))
        check16("e2b backward data", T["g32b"], (T["a2"] > 0) * convT(T["g32a"], po, "e2b"))
        check16("e2a backward data", T["gp1"], convT(T["g32b"], po, "e2a"))
        check16("level 1 pooling gradient", T["g16a"],
                (T["s1"] > 0) * (T["gc1"][:16] + cn.pool2_backward(T["gp1"])))
        check16("e1b backward data", T["g16b"], (T["a1"] > 0) * convT(T["g16a"], po, "e1b"))
        # weight and bias gradients of every layer, from its stored input and
        # the upstream gradient it was given
        for name, a, g in (("out", T["d1"], gy), ("d1b", T["a5"], gz_d1b), ("d1a", cat1, gz_d1a),
                           ("d2b", T["a4"], gz_d2b), ("d2a", cat2, gz_d2a), ("b3b", T["a3"], T["g64a"]),
                           ("b3a", T["p2"], T["g64b"]), ("e2b", T["a2"], T["g32a"]), ("e2a", T["p1"], T["g32b"]),
                           ("e1b", T["a1"], T["g16a"]), ("e1a", T["x"], T["g16b"])):
            gw, gb = wgrad(a, g, po, name)
            ora_g[name + ".w"] += gw
            ora_g[name + ".b"] += gb
    for k in ora_g:
        check("grad " + k, gpu_g[k], ora_g[k])
    print(f"n={n}: worst rel L2 per tensor", {k: f"{v:.1e}" for k, v in worst.items()}, flush=True)
    net.close()
