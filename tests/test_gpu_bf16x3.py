"""The BF16x3 precision policy (PM_F_DFT_BF16X3): the y passes run their
radix-16 stage as dense DFT-16 matrix products on the matrix cores with
split BF16 operands.  Its errors against the FP64 oracle, stated per result:
the 3D transforms, the potential of a solve, and the forces of a whole PM
step of the precision workload's 64^3 sub-run (the same generator with radii
/ 8 and 2^15 particles).  The split keeps about 16 bits of every operand
(2^-16 = 1.5e-5 per product), but only one of the three radix stages of one
of the three axes runs on it, so a transform stays at a few 1e-6 (measured
3.1e-6, FP32: 1-3e-6) and the potential and forces of a whole step at a few
1e-6 (measured 2.9e-6 force, 3.3e-6 potential, FP32: 4e-7): inside the
1e-5 target, about seven times the FP32 path's error.  The measured values
are printed; the bounds sit about three times above them."""
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

from oracle import pm as orc  # noqa: E402
import workloads as W  # noqa: E402
from tests.gpu_util import dev, host, oparams, rel_l2, rel_max, grid, spectrum_array  # noqa: E402


def _log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def M():
    from paper_2312_02968_amd import mondpm
    mondpm.lib()
    return mondpm


@pytest.mark.parametrize("N", [64, 128, 256, 512])
def test_bf16x3_transforms(M, N):
    rng = np.random.default_rng(N + 1)
    x = rng.standard_normal((N, N, N)).astype(np.float32)
    p = dict(W.params(N // 2, n_pad=N), flags=M.PM_F_DFT_BF16X3)
    ctx = M.pm_create(p, 0)
    P = M.pm_spectrum_pitch(N)
    spec = torch.zeros(N * N * P * 2, dtype=torch.float32, device="cuda")
    M.pm_fft_r2c(ctx, dev(x), spec)
    got = spectrum_array(spec, N, P)[:, :, : N // 2 + 1]
    import scipy.fft as sfft
    ref = sfft.rfftn(x.astype(np.float64), workers=orc.WORKERS)
    e_fwd = rel_l2(got, ref)
    out = grid(N)
    M.pm_fft_c2r(ctx, spec, out)
    e_back = rel_l2(host(out).reshape(N, N, N) / N ** 3, x)
    ctx.close()
    _log(f"bf16x3 transform {N}^3: r2c rel L2 {e_fwd:.2e}, c2r(r2c) round trip {e_back:.2e}")
    assert e_fwd < 1e-5 and e_back < 1.5e-5


def test_bf16x3_whole_step_of_the_precision_subrun(M):
    w = W.plummer_mixture(seed=0, N=1 << 15, n=64, a_range=(1.0, 4.0))
    p = dict(w["params"], flags=M.PM_F_DFT_BF16X3)
    n = len(w["mass"])
    op = oparams(w["params"])
    rho_o = orc.deposit(op, w["pos"].astype(np.float64), w["mass"].astype(np.float64))
    phi_o, _ = orc.aqual_solve(op, rho_o)
    acc_o = orc.smooth_accel(op, phi_o, w["pos"].astype(np.float64))
    res = {}
    for name, flags in (("fp32", 0), ("bf16x3", M.PM_F_DFT_BF16X3)):
        ctx = M.pm_create(dict(w["params"], flags=flags), n)
        N = p["n_pad"]
        rho, phi = grid(N), grid(N)
        acc = torch.zeros(3 * n, device="cuda")
        pos = dev(w["pos"])
        M.pm_deposit(ctx, pos, dev(w["mass"]), rho)
        M.aqual_solve(ctx, rho, phi, want_info=False)
        M.smooth_accel(ctx, phi, pos, acc)
        g = host(acc).reshape(-1, 3)
        ph = host(phi).reshape(N, N, N)
        res[name] = dict(phi=rel_l2(ph, phi_o), phi_max=rel_max(ph, phi_o), force=rel_l2(g, acc_o),
                         force_max=rel_max(g, acc_o))
        ctx.close()
    _log("precision sub-run (64^3 grid, 128^3 box, 2^15 particles, K = 4) against the FP64 oracle:",
         {k: {kk: f"{vv:.2e}" for kk, vv in v.items()} for k, v in res.items()})
    assert res["fp32"]["force"] < 1e-5 and res["fp32"]["phi"] < 1e-5
    assert res["bf16x3"]["force"] < 1e-5 and res["bf16x3"]["phi"] < 1e-5
    assert res["bf16x3"]["force_max"] < 2e-5 and res["bf16x3"]["phi_max"] < 2e-5


def test_bf16x3_solve_512(M):
    iso = W.isothermal_sphere(seed=0)
    p0 = dict(iso["params"], iters=2)
    idx = np.random.default_rng(1).choice(len(iso["mass"]), 1 << 14, replace=False)
    m = iso["mass"].astype(np.float64)[idx] * (len(iso["mass"]) / len(idx))
    op = oparams(p0)
    rho = orc.deposit(op, iso["pos"].astype(np.float64)[idx], m).astype(np.float32)
    phi_o, _ = orc.aqual_solve(op, rho.astype(np.float64))
    ctx = M.pm_create(dict(p0, flags=M.PM_F_DFT_BF16X3), 0)
    phi = grid(512)
    M.aqual_solve(ctx, dev(rho), phi, want_info=False)
    got = host(phi).reshape(512, 512, 512)
    e, em = rel_l2(got, phi_o), rel_max(got, phi_o)
    ctx.close()
    _log(f"bf16x3 solve, 256^3 grid in a 512^3 box, K = 2: phi rel L2 {e:.2e}, max {em:.2e}")
    assert e < 1e-5 and em < 2e-5
