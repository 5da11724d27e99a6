"""Helpers for the GPU parity tests: run the HIP path through the C ABI binding
and the FP64 oracle on the same FP32 inputs."""
import numpy as np
import torch

from oracle import pm as orc


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def oparams(d):
    return orc.Params.from_dict(d)


def rel_l2(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    if not (np.iscomplexobj(a) or np.iscomplexobj(b)):
        a, b = a.astype(np.float64), b.astype(np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rel_max(a, b):
    a = np.asarray(a)
    b = np.asarray(b)
    mb = np.max(np.abs(b))
    return float(np.max(np.abs(a - b)) / (mb if mb > 0 else 1.0))


def grid(N):
    return torch.zeros(N ** 3, dtype=torch.float32, device="cuda")
