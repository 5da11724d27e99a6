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
# MONDPM_LIB names another build of the same library (for timing build
# variants side by side); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("MONDPM_LIB") or os.path.join(_HERE, "libmondpm.so")

PM_MU_STANDARD, PM_MU_DEEP, PM_MU_NEWTON = 0, 1, 2
PM_OK, PM_E_INVAL, PM_E_DEVICE, PM_E_NOMEM, PM_E_BOUNDS, PM_E_NOTCONV, PM_E_NONFINITE = 0, -1, -2, -3, -4, -5, -6
PM_F_ANALYTIC_NORM = 0x1
PM_F_RESIDUAL = 0x2
PM_F_WARM_START = 0x4
PM_F_DFT_BF16X3 = 0x8
PM_STORE_FP32 = 0
PM_STORE_FP16 = 1
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
        L.pm_create.argtypes = [P(PmParams), I64, VP, ctypes.c_size_t, VP, P(VP)]
        L.pm_destroy.argtypes = [VP]
        L.pm_deposit.argtypes = [VP, VP, VP, I64, VP]
        L.pm_deposit_noalloc.argtypes = [P(PmParams), VP, VP, I64, VP, VP]
        L.aqual_solve.argtypes = [VP, VP, VP, VP, P(PmSolveInfo)]
        L.smooth_accel.argtypes = [VP, VP, VP, I64, VP]
        L.interp_push.argtypes = [VP, VP, VP, VP, I64, D, D]
        L.pm_step.argtypes = [VP, VP, VP, VP, I64, D, P(PmSolveInfo)]
        L.pm_step_capture.argtypes = [VP, VP, VP, VP, I64, D]
        L.pm_step_replay.argtypes = [VP, ctypes.c_int32]
        L.pm_diagnostics.argtypes = [VP, VP, VP, VP, I64, VP, P(ctypes.c_double)]
        L.pm_spectrum_pitch.argtypes = [ctypes.c_int32]
        L.pm_spectrum_pitch.restype = ctypes.c_int32
        L.pm_fft_r2c.argtypes = [VP, VP, VP]
        L.pm_fft_c2r.argtypes = [VP, VP, VP]
        L.pm_set_timing.argtypes = [VP, ctypes.c_int]
        L.pm_read_timing.argtypes = [VP, P(ctypes.c_double), P(ctypes.c_int64)]
        L.pm_last_error.restype = ctypes.c_char_p
        I32, F32 = ctypes.c_int32, ctypes.c_float
        L.pm_newton_potential.argtypes = [VP, VP, VP]
        L.pm_apparent_density.argtypes = [VP, VP, VP]
        L.pm_set_external_field.argtypes = [VP, D, D, D]
        L.aqual_solve_field.argtypes = [VP, VP, VP, VP, VP, P(PmSolveInfo)]
        L.aqual_solve_increment.argtypes = [VP, VP, VP, VP, I32, VP, VP, P(PmSolveInfo)]
        L.pm_potential_field.argtypes = [VP, VP, VP]
        L.aqual_solve_learned.argtypes = [VP, VP, VP, VP, P(PmSolveInfo)]
        L.pm_net_param_count.argtypes = []
        L.pm_net_param_count.restype = I64
        L.pm_net_create.argtypes = [I32, I32, VP, P(VP)]
        L.pm_net_destroy.argtypes = [VP]
        L.pm_net_set_params.argtypes = [VP, VP]
        L.pm_net_get_params.argtypes = [VP, VP]
        L.pm_net_get_grads.argtypes = [VP, VP]
        L.pm_net_input.argtypes = [VP, VP, VP, I32]
        L.pm_net_target.argtypes = [VP, VP, VP, VP, I32]
        L.pm_net_set_input.argtypes = [VP, I32, VP]
        L.pm_net_get_input.argtypes = [VP, I32, VP]
        L.pm_net_set_target.argtypes = [VP, I32, VP]
        L.pm_net_get_target.argtypes = [VP, I32, VP]
        L.pm_net_run.argtypes = [VP, I32]
        L.pm_net_output.argtypes = [VP, I32, VP]
        L.pm_net_get_tensor.argtypes = [VP, I32, I32, VP]
        L.pm_net_get_rms.argtypes = [VP, I32, P(D)]
        L.pm_net_backward.argtypes = [VP, I32, P(D)]
        L.pm_net_adam.argtypes = [VP, F32]
        L.pm_net_train_step.argtypes = [VP, I32, F32, P(D)]
        L.pm_net_forward.argtypes = [VP, VP, VP, VP]
        for f in ("pm_create", "pm_destroy", "pm_deposit", "pm_deposit_noalloc", "aqual_solve", "smooth_accel", "interp_push",
                  "pm_step", "pm_step_capture", "pm_step_replay", "pm_diagnostics", "pm_fft_r2c", "pm_fft_c2r", "pm_set_timing",
                  "pm_read_timing", "pm_newton_potential", "pm_apparent_density", "pm_set_external_field", "aqual_solve_field", "pm_net_create",
                  "pm_net_destroy", "pm_net_set_params", "pm_net_get_params", "pm_net_get_grads",
                  "pm_net_input", "pm_net_target", "pm_net_set_input", "pm_net_get_input",
                  "pm_net_set_target", "pm_net_get_target", "pm_net_run", "pm_net_output", "pm_net_get_tensor", "pm_net_get_rms",
                  "pm_net_backward", "pm_net_adam", "pm_net_train_step", "pm_net_forward"):
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
    """Owns a pm_ctx bound to a stream.  By default its workspace is a torch
    tensor (caller-owned device memory, as the C ABI expects); with
    workspace="library" the library allocates it instead."""

    def __init__(self, params, max_particles=0, stream=None, workspace="torch"):
        self.params = dict(params)
        self._p = make_params(params)
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.workspace = None
        ws_ptr, ws_bytes = None, 0
        if workspace == "torch":
            ws_bytes = int(lib().pm_workspace_bytes(ctypes.byref(self._p), int(max_particles)))
            if ws_bytes == 0:
                _check(PM_E_INVAL, "pm_workspace_bytes")
            # 256 spare bytes to align the start
            self.workspace = torch.empty(ws_bytes + 256, dtype=torch.uint8, device="cuda")
            base = self.workspace.data_ptr()
            ws_ptr = ctypes.c_void_p((base + 255) & ~255)
        elif workspace != "library":
            raise ValueError("workspace must be 'torch' or 'library'")
        h = ctypes.c_void_p()
        _check(lib().pm_create(ctypes.byref(self._p), int(max_particles), ws_ptr, ws_bytes,
                               ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)), "pm_create")
        self.handle = h
        self.max_particles = int(max_particles)
        self.N = int(params["n_pad"])

    def close(self):
        if getattr(self, "handle", None):
            lib().pm_destroy(self.handle)
            self.handle = None
        self.workspace = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pm_create(params, max_particles=0, stream=None, workspace="torch") -> Ctx:
    return Ctx(params, max_particles, stream, workspace)


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


def pm_deposit_noalloc(params, pos, mass, rho, stream=None):
    """pm_deposit without a context or any device allocation (fixed scratch)."""
    n = mass.numel()
    p = make_params(params)
    if stream is None:
        stream = torch.cuda.current_stream()
    _check(lib().pm_deposit_noalloc(ctypes.byref(p), _ptr(pos, numel=3 * n, name="pos"), _ptr(mass, name="mass"),
                                    n, _ptr(rho, numel=int(params["n_pad"]) ** 3, name="rho"),
                                    ctypes.c_void_p(stream.cuda_stream)), "pm_deposit_noalloc")
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


def pm_step_capture(ctx: Ctx, pos, vel, mass, dt):
    """Records one pm_step on these buffers as a graph kept by the context
    (nothing runs); the context must live on a created stream."""
    n = mass.numel()
    _check(lib().pm_step_capture(ctx.handle, _ptr(pos, numel=3 * n, name="pos"),
                                 _ptr(vel, numel=3 * n, name="vel"), _ptr(mass, name="mass"), n, float(dt)),
           "pm_step_capture")


def pm_step_replay(ctx: Ctx, count=1):
    _check(lib().pm_step_replay(ctx.handle, int(count)), "pm_step_replay")


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


# ---------------------------------------------------------------------------
# Newton potential, field solve and the learned start
# ---------------------------------------------------------------------------

def pm_newton_potential(ctx: Ctx, rho, phiN):
    R = ctx.N ** 3
    _check(lib().pm_newton_potential(ctx.handle, _ptr(rho, numel=R, name="rho"), _ptr(phiN, numel=R, name="phiN")),
           "pm_newton_potential")
    return phiN


def pm_apparent_density(ctx: Ctx, phi, rho_a):
    R = ctx.N ** 3
    _check(lib().pm_apparent_density(ctx.handle, _ptr(phi, numel=R, name="phi"), _ptr(rho_a, numel=R, name="rho_a")),
           "pm_apparent_density")
    return rho_a


def pm_set_external_field(ctx: Ctx, g):
    """Uniform external Newtonian field g = (gx, gy, gz) for later solves on ctx."""
    gx, gy, gz = (float(v) for v in g)
    _check(lib().pm_set_external_field(ctx.handle, gx, gy, gz), "pm_set_external_field")


def aqual_solve_field(ctx: Ctx, rho, phi, F, H0=None, want_info=True):
    R = ctx.N ** 3
    info = PmSolveInfo()
    _check(lib().aqual_solve_field(ctx.handle, _ptr(rho, numel=R, name="rho"),
                                   _ptr(H0, numel=3 * R, name="H0"), _ptr(phi, numel=R, name="phi"),
                                   _ptr(F, numel=3 * R, name="F"),
                                   ctypes.byref(info) if want_info else None), "aqual_solve_field")
    return info.to_dict() if want_info else None


def aqual_solve_increment(ctx: Ctx, d_rho, F, gM, d_phi, storage=PM_STORE_FP16, d_F=None, want_info=True):
    """Linearised increment solve (see include/mondpm.h): d_phi from d_rho
    about the previous F and g_M, with FP16 (default) or FP32 spectra."""
    R = ctx.N ** 3
    info = PmSolveInfo()
    _check(lib().aqual_solve_increment(ctx.handle, _ptr(d_rho, numel=R, name="d_rho"),
                                       _ptr(F, numel=3 * R, name="F"), _ptr(gM, numel=3 * R, name="gM"),
                                       int(storage), _ptr(d_phi, numel=R, name="d_phi"),
                                       _ptr(d_F, numel=3 * R, name="d_F"),
                                       ctypes.byref(info) if want_info else None), "aqual_solve_increment")
    return info.to_dict() if want_info else None


def pm_potential_field(ctx: Ctx, phi, g):
    """g = -i kt phi_hat on the FFT box (the field of phi as the curl-free
    projection forms it)."""
    R = ctx.N ** 3
    _check(lib().pm_potential_field(ctx.handle, _ptr(phi, numel=R, name="phi"), _ptr(g, numel=3 * R, name="g")),
           "pm_potential_field")


def aqual_solve_learned(ctx: Ctx, net, rho, phi, want_info=True):
    """aqual_solve from the learned start of net in one call (see
    include/mondpm.h)."""
    info = PmSolveInfo()
    _check(lib().aqual_solve_learned(ctx.handle, net.handle, _ptr(rho, numel=ctx.N ** 3, name="rho"),
                                     _ptr(phi, numel=ctx.N ** 3, name="phi"),
                                     ctypes.byref(info) if want_info else None), "aqual_solve_learned")
    return info.to_dict() if want_info else None


def pm_net_param_count() -> int:
    return int(lib().pm_net_param_count())


class Net:
    """Owns a pm_net (learned-start network) bound to a stream."""

    def __init__(self, n, max_batch=1, stream=None):
        if stream is None:
            stream = torch.cuda.current_stream()
        self.stream = stream
        self.n = int(n)
        self.max_batch = int(max_batch)
        h = ctypes.c_void_p()
        _check(lib().pm_net_create(self.n, self.max_batch, ctypes.c_void_p(stream.cuda_stream), ctypes.byref(h)),
               "pm_net_create")
        self.handle = h

    def close(self):
        if getattr(self, "handle", None):
            lib().pm_net_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def pm_net_create(n, max_batch=1, stream=None) -> Net:
    return Net(n, max_batch, stream)


def pm_net_destroy(net: Net):
    net.close()


def _host_f32(a, count, name):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32).reshape(-1)
    if a.size != count:
        raise ValueError(f"{name} has {a.size} elements, needs {count}")
    return a


def pm_net_set_params(net: Net, params):
    P = pm_net_param_count()
    a = _host_f32(params, P, "params")
    _check(lib().pm_net_set_params(net.handle, a.ctypes.data_as(ctypes.c_void_p)), "pm_net_set_params")


def pm_net_get_params(net: Net):
    import numpy as np
    a = np.empty(pm_net_param_count(), dtype=np.float32)
    _check(lib().pm_net_get_params(net.handle, a.ctypes.data_as(ctypes.c_void_p)), "pm_net_get_params")
    return a


def pm_net_get_grads(net: Net):
    import numpy as np
    a = np.empty(pm_net_param_count(), dtype=np.float32)
    _check(lib().pm_net_get_grads(net.handle, a.ctypes.data_as(ctypes.c_void_p)), "pm_net_get_grads")
    return a


def pm_net_input(ctx: Ctx, net: Net, phiN, slot=0):
    _check(lib().pm_net_input(ctx.handle, net.handle, _ptr(phiN, numel=ctx.N ** 3, name="phiN"), int(slot)),
           "pm_net_input")


def pm_net_target(ctx: Ctx, net: Net, phiN, F, slot=0):
    R = ctx.N ** 3
    _check(lib().pm_net_target(ctx.handle, net.handle, _ptr(phiN, numel=R, name="phiN"),
                               _ptr(F, numel=3 * R, name="F"), int(slot)), "pm_net_target")


def pm_net_set_input(net: Net, slot, x):
    _check(lib().pm_net_set_input(net.handle, int(slot), _ptr(x, numel=4 * net.n ** 3, name="x")),
           "pm_net_set_input")


def pm_net_get_input(net: Net, slot, x):
    _check(lib().pm_net_get_input(net.handle, int(slot), _ptr(x, numel=4 * net.n ** 3, name="x")),
           "pm_net_get_input")
    return x


def pm_net_set_target(net: Net, slot, y):
    _check(lib().pm_net_set_target(net.handle, int(slot), _ptr(y, numel=3 * net.n ** 3, name="y")),
           "pm_net_set_target")


def pm_net_get_target(net: Net, slot, y):
    _check(lib().pm_net_get_target(net.handle, int(slot), _ptr(y, numel=3 * net.n ** 3, name="y")),
           "pm_net_get_target")
    return y


def pm_net_run(net: Net, batch=1):
    _check(lib().pm_net_run(net.handle, int(batch)), "pm_net_run")


def pm_net_output(net: Net, slot, y):
    _check(lib().pm_net_output(net.handle, int(slot), _ptr(y, numel=3 * net.n ** 3, name="y")), "pm_net_output")
    return y


# tensors of pm_net_get_tensor: name -> (index, channels, level)
NET_TENSORS = {
    "x": (0, 4, 0), "a1": (1, 16, 0), "s1": (2, 16, 0), "p1": (3, 16, 1), "a2": (4, 32, 1),
    "s2": (5, 32, 1), "p2": (6, 32, 2), "a3": (7, 64, 2), "b3": (8, 64, 2), "a4": (9, 32, 1),
    "d2": (10, 32, 1), "a5": (11, 16, 0), "d1": (12, 16, 0),
    "g16a": (13, 16, 0), "g16b": (14, 16, 0), "gc1": (15, 48, 0), "g32a": (16, 32, 1), "g32b": (17, 32, 1),
    "gc2": (18, 96, 1), "g64a": (19, 64, 2), "g64b": (20, 64, 2), "gp1": (21, 16, 1), "gp2": (22, 32, 2),
}


def pm_net_get_tensor(net: Net, name, slot=0):
    """A stored activation or gradient tensor as a CUDA tensor [C, m, m, m]."""
    which, C, level = NET_TENSORS[name]
    m = net.n >> level
    out = torch.empty(C * m ** 3, device="cuda")
    _check(lib().pm_net_get_tensor(net.handle, int(which), int(slot), _ptr(out)), "pm_net_get_tensor")
    return out.view(C, m, m, m)


def pm_net_get_rms(net: Net, slot=0) -> float:
    r = ctypes.c_double()
    _check(lib().pm_net_get_rms(net.handle, int(slot), ctypes.byref(r)), "pm_net_get_rms")
    return r.value


def pm_net_backward(net: Net, batch=1, want_loss=True):
    loss = ctypes.c_double()
    _check(lib().pm_net_backward(net.handle, int(batch), ctypes.byref(loss) if want_loss else None),
           "pm_net_backward")
    return loss.value if want_loss else None


def pm_net_adam(net: Net, lr):
    _check(lib().pm_net_adam(net.handle, float(lr)), "pm_net_adam")


def pm_net_train_step(net: Net, batch, lr, want_loss=True):
    loss = ctypes.c_double()
    _check(lib().pm_net_train_step(net.handle, int(batch), float(lr), ctypes.byref(loss) if want_loss else None),
           "pm_net_train_step")
    return loss.value if want_loss else None


def pm_net_forward(ctx: Ctx, net: Net, phiN, H0):
    R = ctx.N ** 3
    _check(lib().pm_net_forward(ctx.handle, net.handle, _ptr(phiN, numel=R, name="phiN"),
                                _ptr(H0, numel=3 * R, name="H0")), "pm_net_forward")
    return H0
