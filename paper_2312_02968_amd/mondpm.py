"""Thin Python binding of libmondpm.so (include/mondpm.h).

The functions carry the names of the C entry points and only marshal
arguments: torch CUDA tensors become device pointers, parameter dictionaries
become ``pm_params``.  Every computation runs in the HIP library.  Loading
fails loudly when the library has not been built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmondpm.so")

PM_MU_STANDARD, PM_MU_DEEP, PM_MU_NEWTON = 0, 1, 2
PM_OK, PM_E_INVAL, PM_E_DEVICE, PM_E_NOMEM, PM_E_BOUNDS, PM_E_NOTCONV, PM_E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
PM_F_ANALYTIC_NORM = 0x1
PM_F_RESIDUAL = 0x2
TIMERS = ["x_fwd_real", "x_fwd_real3", "x_inv_real", "x_nu", "x_mu", "y_fwd", "y_inv", "z_fwd",
          "z_inv", "z_newton", "z_curl", "z_curl_final", "z_div", "sort", "deposit", "gather", "fill",
          "reduce"]


class PmParams(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("n_pad", ctypes.c_int32), ("box", ctypes.c_double),
                ("G", ctypes.c_double), ("a0", ctypes.c_double), ("mu", ctypes.c_int32),
                ("sigma", ctypes.c_double), ("cutoff", ctypes.c_double), ("iters", ctypes.c_int32),
                ("tol", ctypes.c_double), ("flags", ctypes.c_uint32)]


class PmSolveInfo(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("status", ctypes.c_int32),
                ("n_residuals", ctypes.c_int32), ("bounds_flag", ctypes.c_int32),
                ("residual", ctypes.c_double * 64), ("gN_norm", ctypes.c_double)]

    def to_dict(self):
        return dict(iterations=self.iterations, status=self.status, bounds_flag=self.bounds_flag,
                    residuals=[self.residual[i] for i in range(self.n_residuals)],
                    gN_norm=self.gN_norm)


_lib = None


def lib():
    """The loaded library; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python -m paper_2312_02968_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        P, VP, I64, D = ctypes.POINTER, ctypes.c_void_p, ctypes.c_int64, ctypes.c_double
        L.pm_workspace_bytes.argtypes = [P(PmParams), I64]
        L.pm_workspace_bytes.restype = ctypes.c_size_t
        L.pm_create.argtypes = [P(PmParams), I64, VP, P(VP)]
        L.pm_destroy.argtypes = [VP]
        L.pm_deposit.argtypes = [VP, VP, VP, I64, VP]
        L.aqual_solve.argtypes = [VP, VP, VP, VP, P(PmSolveInfo)]
        L.smooth_accel.argtypes = [VP, VP, VP, I64, VP]
        L.interp_push.argtypes = [VP, VP, VP, VP, I64, D, D]
        L.pm_step.argtypes = [VP, VP, VP, VP, I64, D, P(PmSolveInfo)]
        L.pm_diagnostics.argtypes = [VP, VP, VP, VP, I64, VP, P(ctypes.c_double)]
        L.pm_spectrum_pitch.argtypes = [ctypes.c_int32]
        L.pm_spectrum_pitch.restype = ctypes.c_int32
        L.pm_fft_r2c.argtypes = [VP, VP, VP]
        L.pm_fft_c2r.argtypes = [VP, VP, VP]
        L.pm_set_timing.argtypes = [VP, ctypes.c_int]
        L.pm_read_timing.argtypes = [VP, P(ctypes.c_double), P(ctypes.c_int64)]
        L.pm_last_error.restype = ctypes.c_char_p
        for f in ("pm_create", "pm_destroy", "pm_deposit", "aqual_solve", "smooth_accel", "interp_push",
                  "pm_step", "pm_diagnostics", "pm_fft_r2c", "pm_fft_c2r", "pm_set_timing",
                  "pm_read_timing"):
            getattr(L, f).restype = ctypes.c_int
        _lib = L
    return _lib


class PmError(RuntimeError):
    def __init__(self, status, where):
        msg = lib().pm_last_error().decode(errors="replace")
        super().__init__(f"{where} failed with status {status}: {msg}")
        self.status = status


def _check(status, where):
    if status != PM_OK:
        raise PmError(status, where)


def make_params(d) -> PmParams:
    return PmParams(int(d["n"]), int(d["n_pad"]), float(d["box"]), float(d.get("G", 1.0)),
                    float(d.get("a0", 1.0)), int(d.get("mu", 0)), float(d.get("sigma", 1.0)),
                    float(d.get("cutoff", 4.0)), int(d.get("iters", 4)), float(d.get("tol", 0.0)),
                    int(d.get("flags", 0)))


def _ptr(t, dtype=torch.float32, numel=None, name="tensor"):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return ctypes.c_void_p(t.data_ptr())


class Ctx:
    """Owns a pm_ctx (device workspace) bound to a stream."""

    def __init__(self, params, max_particles=0, stream=None):
        self.params = dict(params)
        self._p = make_params(params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        h = ctypes.c_void_p()
        _check(lib().pm_create(ctypes.byref(self._p), int(max_particles),
                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), "pm_create")
        self.handle = h
        self.max_particles = int(max_particles)
        self.N = int(params["n_pad"])

    def close(self):
        if getattr(self, "handle", None):
            lib().pm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pm_create(params, max_particles=0, stream=None) -> Ctx:
    return Ctx(params, max_particles, stream)


def pm_destroy(ctx: Ctx):
    ctx.close()


def pm_workspace_bytes(params, max_particles=0) -> int:
    p = make_params(params)
    return int(lib().pm_workspace_bytes(ctypes.byref(p), int(max_particles)))


def pm_spectrum_pitch(n_pad) -> int:
    return int(lib().pm_spectrum_pitch(int(n_pad)))


def pm_deposit(ctx: Ctx, pos, mass, rho):
    n = mass.numel()
    _check(lib().pm_deposit(ctx.handle, _ptr(pos, numel=3 * n, name="pos"), _ptr(mass, name="mass"), n,
                            _ptr(rho, numel=ctx.N ** 3, name="rho")), "pm_deposit")
    return rho


def aqual_solve(ctx: Ctx, rho, phi, H0=None, want_info=True):
    info = PmSolveInfo()
    _check(lib().aqual_solve(ctx.handle, _ptr(rho, numel=ctx.N ** 3, name="rho"),
                             _ptr(H0, numel=3 * ctx.N ** 3, name="H0"),
                             _ptr(phi, numel=ctx.N ** 3, name="phi"),
                             ctypes.byref(info) if want_info else None), "aqual_solve")
    return info.to_dict() if want_info else None


def smooth_accel(ctx: Ctx, phi, pos, acc):
    n = pos.numel() // 3
    _check(lib().smooth_accel(ctx.handle, _ptr(phi, numel=ctx.N ** 3, name="phi"), _ptr(pos, name="pos"), n,
                              _ptr(acc, numel=3 * n, name="acc")), "smooth_accel")
    return acc


def interp_push(ctx: Ctx, phi, pos, vel, dt_kick, dt_drift):
    n = pos.numel() // 3
    _check(lib().interp_push(ctx.handle, _ptr(phi, numel=ctx.N ** 3, name="phi"), _ptr(pos, name="pos"),
                             _ptr(vel, numel=3 * n, name="vel"), n, float(dt_kick), float(dt_drift)),
           "interp_push")


def pm_step(ctx: Ctx, pos, vel, mass, dt, want_info=False):
    n = mass.numel()
    info = PmSolveInfo()
    _check(lib().pm_step(ctx.handle, _ptr(pos, numel=3 * n, name="pos"), _ptr(vel, numel=3 * n, name="vel"),
                         _ptr(mass, name="mass"), n, float(dt),
                         ctypes.byref(info) if want_info else None), "pm_step")
    return info.to_dict() if want_info else None


def pm_diagnostics(ctx: Ctx, pos, vel, mass, phi=None):
    n = mass.numel()
    out = (ctypes.c_double * 10)()
    _check(lib().pm_diagnostics(ctx.handle, _ptr(pos, numel=3 * n, name="pos"),
                                _ptr(vel, numel=3 * n, name="vel"), _ptr(mass, name="mass"), n,
                                _ptr(phi, numel=ctx.N ** 3, name="phi"), out), "pm_diagnostics")
    v = list(out)
    return dict(P=v[0:3], L=v[3:6], Ekin=v[6], mass=v[7], Epot_sum=v[8], out_of_region=int(v[9]))


def pm_fft_r2c(ctx: Ctx, real, spec):
    """spec: float32 tensor of n_pad * n_pad * pitch * 2 elements (complex pairs)."""
    _check(lib().pm_fft_r2c(ctx.handle, _ptr(real, numel=ctx.N ** 3, name="real"),
                            _ptr(spec, numel=2 * ctx.N * ctx.N * pm_spectrum_pitch(ctx.N), name="spec")),
           "pm_fft_r2c")
    return spec


def pm_fft_c2r(ctx: Ctx, spec, real):
    _check(lib().pm_fft_c2r(ctx.handle, _ptr(spec, numel=2 * ctx.N * ctx.N * pm_spectrum_pitch(ctx.N),
                                             name="spec"),
                            _ptr(real, numel=ctx.N ** 3, name="real")), "pm_fft_c2r")
    return real


def pm_set_timing(ctx: Ctx, enable: bool):
    _check(lib().pm_set_timing(ctx.handle, 1 if enable else 0), "pm_set_timing")


def pm_read_timing(ctx: Ctx):
    """{timer name: (total ms, launches)} recorded with HIP events since the last read."""
    n = len(TIMERS)
    ms = (ctypes.c_double * n)()
    cnt = (ctypes.c_int64 * n)()
    _check(lib().pm_read_timing(ctx.handle, ms, cnt), "pm_read_timing")
    return {TIMERS[i]: (ms[i], cnt[i]) for i in range(n) if cnt[i] > 0}
