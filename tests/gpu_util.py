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


def spectrum_array(spec, N, P):
    """Complex [kz][ky][kx] array (kx < P) of a spectrum in the library's grouped
    layout [kx / 16][kz][ky][kx % 16] (float pairs)."""
    s = host(spec).reshape(P // 16, N, N, 16, 2).transpose(1, 2, 0, 3, 4).reshape(N, N, P, 2)
    return s[..., 0] + 1j * s[..., 1]


def spectrum_tensor(arr, N, P):
    """Inverse of spectrum_array: a complex [kz][ky][kx < P] array as a device
    tensor in the grouped layout."""
    a = np.zeros((N, N, P, 2), dtype=np.float32)
    a[..., 0] = arr.real
    a[..., 1] = arr.imag
    g = a.reshape(N, N, P // 16, 16, 2).transpose(2, 0, 1, 3, 4)
    return torch.from_numpy(np.ascontiguousarray(g).reshape(-1)).cuda()
