"""pm_deposit_noalloc (the deposit for callers that cannot allocate) against
pm_deposit on a context, through the C ABI: two calls in a row, the second
with a smaller input, each to the density bar of the parity tests (1e-6 of
the largest cell; both sum their cells with atomic adds in no fixed order)."""
import numpy as np
import pytest
import torch

import workloads as W
from paper_2312_02968_amd import mondpm as M

pytestmark = pytest.mark.gpu


def _case(seed, n, N, sigma):
    w = W.random_cloud(seed, n, N, mu=W.MU_STANDARD, sigma=sigma)
    return w["params"], w["pos"], w["mass"]


def test_noalloc_deposit_matches_pm_deposit_twice():
    cases = [_case(5, 64, 20000, 1.0), _case(6, 16, 300, 1.5)]    # the second smaller
    for p, pos, mass in cases:
        N = p["n_pad"]
        print(f"noalloc case n_pad={N} particles={len(mass)} sigma={p['sigma']}", flush=True)
        pos_d = torch.from_numpy(pos).cuda()
        mass_d = torch.from_numpy(mass).cuda()
        rho_a = torch.full((N ** 3,), 7.0, device="cuda")         # overwritten by the call
        M.pm_deposit_noalloc(p, pos_d, mass_d, rho_a)
        ctx = M.pm_create(p, len(mass))
        rho_b = torch.empty(N ** 3, device="cuda")
        M.pm_deposit(ctx, pos_d, mass_d, rho_b)
        torch.cuda.synchronize()
        a, b = rho_a.cpu().numpy(), rho_b.cpu().numpy()
        ctx.close()
        assert np.max(np.abs(a - b)) <= 1e-6 * np.max(np.abs(b)), np.max(np.abs(a - b))
        assert abs(a.sum() - b.sum()) <= 1e-5 * abs(b.sum())


def test_noalloc_rejects_sizes_beyond_its_scratch():
    import ctypes as C
    one = torch.zeros(16, device="cuda")
    ptr = C.c_void_p(one.data_ptr())
    big = M.make_params(W.params(512))                       # n_pad 1024 > 512
    assert M.lib().pm_deposit_noalloc(C.byref(big), ptr, ptr, 4, ptr, None) == M.PM_E_INVAL
    small = M.make_params(W.params(16))
    assert M.lib().pm_deposit_noalloc(C.byref(small), ptr, ptr, (1 << 20) + 1, ptr, None) == M.PM_E_INVAL
