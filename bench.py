"""Throughput of the MOND particle-mesh step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload isothermal]
                    [--no-cpu-baseline] [--no-oracle-error]

Runs W untimed and K timed PM steps (deposit, AQUAL solve with 4 iterations,
gather, kick and drift) through the C ABI on the default workload: the
self-consistent isothermal sphere of 2^20 equal masses on a 256^3 grid in a
512^3 periodic FFT box (standard interpolation, sigma = 1 cell).  Inputs are
resident in HBM before the timed region.  Prints one JSON line.

The timed region is K replays of the step recorded once as a HIP graph
(pm_step_capture / pm_step_replay; --launch eager times K pm_step calls
instead).  K eager steps follow with a HIP event pair around every launch on
the library's stream: they give the per-kernel durations of the roofline
record, for the kernel with the largest share of the step, and their own
ms/step.  The line also carries a CPU baseline (the FP64 oracle timed on a
bounded sample of the same workload on the host cores) and, for FFT boxes up
to 512^3, the configuration's force error against the FP64 oracle on the
same input.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "PM steps/s at 256³ grid, 2^20 particles; learned vs plain solve time at 1e-5 res"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_counters.json")
KERNEL_SOURCES = ("paper_2312_02968_amd/csrc/pm_fft.hip", "paper_2312_02968_amd/csrc/pm_device.h",
                  "paper_2312_02968_amd/csrc/pm_particles.hip", "paper_2312_02968_amd/csrc/pm_pieces.hip")


def source_hash():
    """Hash of the kernel sources, to tell whether stored counters still apply."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE x fetch_scale + WRITE_SIZE x write_scale), or None when the
    summary is missing, was taken on different kernel sources or on another
    workload."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if (t.get("source_hash") != source_hash() or t.get("workload") != workload
            or kernel not in t.get("kernels", {})):
        return None
    return t["kernels"][kernel]["bytes_per_launch"]


_X_MODES = {0: "x_fwd_real", 1: "x_inv_real", 2: "x_nu", 3: "x_mu", 4: "x_nu_keep", 5: "x_lin_nu", 6: "x_lin_nu_keep",
            7: "x_lin_mu", 8: "x_fwd_coarse3"}
_Z_OPS = {0: "z_fwd", 1: "z_inv", 2: "z_newton", 3: "z_curl", 4: "z_curl_final", 5: "z_div", 6: "z_newton",
          7: "z_poisson", 8: "z_newton", 9: "z_apparent", 10: "z_grad", 11: "z_newton", 12: "z_poisson"}


def timer_name(kernel):
    """The library's timer name for an FFT-pass kernel symbol as rocprofv3
    prints it (the timers of the roofline record); passes that read or write
    FP16 spectra get the suffix "_h", torch's own kernels the prefix "torch:",
    other kernels keep their base name."""
    import re
    if "at::native::" in kernel:
        m3 = re.search(r"at::native::([A-Za-z0-9_]+)", kernel)
        return "torch:" + m3.group(1)
    m = re.search(r"(k_[a-z0-9_]+)<([^>]*)>", kernel)
    if not m:
        m2 = re.search(r"(k_[a-z0-9_]+|__amd_rocclr_[A-Za-z]+)", kernel)
        return m2.group(1) if m2 else kernel.split("(")[0].strip()
    base, args = m.group(1), [t.strip() for t in m.group(2).split(",")]
    half = lambda name, io: name + "_h" if int(io) else name
    if base == "k_ypass":                   # <L, T, NT, INV, IO>
        return half("y_inv" if args[3] == "true" else "y_fwd", args[4])
    if base == "k_ypass_mfma":              # <L, INV>
        return "y_inv" if args[1] == "true" else "y_fwd"
    if base == "k_xpass_wave":              # <H, XMODE, NC, IO>
        mode, nc, io = int(args[1]), int(args[2]), args[3]
    elif base == "k_xpass":                 # <H, ROWS, NC, NT, XMODE, IO>
        mode, nc, io = int(args[4]), int(args[2]), args[5]
    elif base == "k_zpass":                 # <L, T, NT, HZ, ZOP, IO>
        return half(_Z_OPS.get(int(args[4]), base), args[5])
    else:
        return base
    name = _X_MODES.get(mode, base)
    return half(name + "3" if name == "x_fwd_real" and nc == 3 else name, io)


def _counter_means(path, counter, K=None):
    """{kernel timer name: (mean counter value per dispatch, dispatches)} from
    a rocprofv3 --pmc CSV (rows of one dispatch are summed first).  With K,
    the y passes (launched with three field components 2K - 1 times per PM
    step and with one component once) are averaged in that mix, as the
    algorithmic bytes per launch are."""
    import csv
    import glob
    from collections import defaultdict
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {path}")
    per_disp = defaultdict(float)
    name_of = {}
    grid_of = {}
    for fn in files:
        for r in csv.DictReader(open(fn)):
            if r["Counter_Name"] != counter:
                continue
            d = (fn, r["Dispatch_Id"])
            per_disp[d] += float(r["Counter_Value"])
            name_of[d] = timer_name(r["Kernel_Name"])
            grid_of[d] = int(r["Grid_Size"])
    acc = defaultdict(lambda: defaultdict(list))
    for d, v in per_disp.items():
        acc[name_of[d]][grid_of[d]].append(v)
    out = {}
    for k, by_grid in acc.items():
        n = sum(len(v) for v in by_grid.values())
        if K and k in ("y_fwd", "y_inv") and len(by_grid) == 2:
            g1, g3 = sorted(by_grid)
            m1 = sum(by_grid[g1]) / len(by_grid[g1])
            m3 = sum(by_grid[g3]) / len(by_grid[g3])
            out[k] = ((2 * K - 1) * m3 + m1) / (2 * K), n
        else:
            allv = [x for v in by_grid.values() for x in v]
            out[k] = sum(allv) / len(allv), n
    return out


def ingest_counters(root, workload, src_hash, K):
    """Write profiles/traffic_counters.json from four rocprofv3 --pmc runs under
    root: FETCH_SIZE and WRITE_SIZE of the bench command, and of the copy
    probe (FETCH_SIZE_copy, WRITE_SIZE_copy), which fixes the KiB-to-bytes
    scale of each counter (HBM bytes = FETCH x fetch_scale + WRITE x
    write_scale, in KiB)."""
    fetch = _counter_means(os.path.join(root, "FETCH_SIZE"), "FETCH_SIZE", K)
    write = _counter_means(os.path.join(root, "WRITE_SIZE"), "WRITE_SIZE", K)
    cf = _counter_means(os.path.join(root, "FETCH_SIZE_copy"), "FETCH_SIZE")
    cw = _counter_means(os.path.join(root, "WRITE_SIZE_copy"), "WRITE_SIZE")
    copy_kib = 1024.0 * 1024.0                   # one 1 GiB copy per dispatch
    kc = "__amd_rocclr_copyBuffer"
    fs = round(copy_kib / max(cf[kc][0], 1.0), 2)
    ws = round(copy_kib / max(cw[kc][0], 1.0), 2)
    kern = {}
    for k in sorted(set(fetch) | set(write)):
        fk = fetch.get(k, (0.0, 0))[0]
        wk = write.get(k, (0.0, 0))[0]
        kern[k] = {"fetch_kib": round(fk, 1), "write_kib": round(wk, 1),
                   "bytes_per_launch": int(1024 * (fk * fs + wk * ws)),
                   "dispatches": max(fetch.get(k, (0, 0))[1], write.get(k, (0, 0))[1])}
    out = {"source_hash": src_hash, "workload": workload, "fetch_scale": fs, "write_scale": ws,
           "copy_probe_kib": {"fetch": cf[kc][0], "write": cw[kc][0]}, "kernels": kern}
    with open(TRAFFIC_FILE, "w") as f:
        json.dump(out, f, indent=1)
    for k, v in sorted(kern.items(), key=lambda kv: -kv[1]["bytes_per_launch"]):
        print(f"{k:24s} {v['fetch_kib']:12.0f} {v['write_kib']:12.0f} {v['bytes_per_launch'] / 1e9:8.3f} GB")


def copy_probe():
    """A plain device copy of known size (1 GiB, three times): the reference
    that scales the HBM byte counters."""
    import torch
    a = torch.empty(256 * 1024 * 1024, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(3):
        b.copy_(a)
    torch.cuda.synchronize()
    print("copy probe: 3 x 1 GiB device copy done", flush=True)


def fft_compare(n_pad=512, reps=20):
    """Times this library's real 3D transforms (pm_fft_r2c / pm_fft_c2r) beside
    torch.fft.rfftn / irfftn (rocFFT) on the same n_pad^3 FP32 input, for
    context only; prints one JSON line."""
    import torch
    from paper_2312_02968_amd import mondpm as M
    import workloads as W
    p = W.params(n_pad // 2, n_pad=n_pad)
    ctx = M.pm_create(p, 0)
    g = torch.Generator(device="cpu").manual_seed(0)
    x = torch.randn(n_pad ** 3, generator=g).cuda()
    spec = torch.empty(2 * n_pad * n_pad * M.pm_spectrum_pitch(n_pad), device="cuda")
    back = torch.empty_like(x)
    x3 = x.view(n_pad, n_pad, n_pad)

    def timed(fn):
        for _ in range(3):
            fn()
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        s.record()
        for _ in range(reps):
            fn()
        e.record()
        torch.cuda.synchronize()
        return s.elapsed_time(e) / reps

    res = {"n_pad": n_pad, "reps": reps,
           "pm_r2c_ms": timed(lambda: M.pm_fft_r2c(ctx, x, spec)),
           "pm_c2r_ms": timed(lambda: M.pm_fft_c2r(ctx, spec, back))}
    xs = torch.fft.rfftn(x3)
    res["rocfft_r2c_ms"] = timed(lambda: torch.fft.rfftn(x3))
    res["rocfft_c2r_ms"] = timed(lambda: torch.fft.irfftn(xs, s=x3.shape))
    ctx.close()
    print(json.dumps({k: (round(v, 4) if isinstance(v, float) else v) for k, v in res.items()}), flush=True)


def start_comparison(w):
    """Learned start (committed weights) and warm start against the zero start
    on the same workload, outside the timed region: potential error against a
    30-iteration reference, iterations to the accuracy of the plain 4-iteration
    solve, wall times, and the warm start's error and step time along a
    10-step trajectory."""
    from paper_2312_02968_amd import learned as L
    from paper_2312_02968_amd import mondpm as M
    res = {}
    fb = L.DEFAULT_FACTOR
    wpath = L.weights_for(fb)
    if os.path.exists(wpath):
        net = M.Net(w["params"]["n_pad"] // fb, 1)
        M.pm_net_set_params(net, L.load_params(wpath))
        r = L.compare_starts(w, net)
        keep = ("K_plain", "K_learned", "plain_err", "learned_err", "t_plain_ms", "t_learned_ms", "t_start_ms",
                "tol", "tol_iters_plain", "tol_iters_learned", "t_tol_plain_ms", "t_tol_learned_ms",
                "tol_fixed_point_diff", "tol_fallback")
        res["learned_start"] = dict({k: r[k] for k in keep}, factor=fb)
        # the metric's residual 1e-5 on the held-out inputs of the workload's
        # size: 16 Plummer mixtures and the isothermal sphere, which stalls
        # above 1e-5 (its learned solve falls back to the zero start)
        if w["params"]["n"] == 256:
            rows = [L.compare_starts(x, net, tol=1e-5) for x in L.held_out_inputs(256, 16)]
            res["learned_start_1e-5"] = dict(L.summarize(rows), factor=fb,
                                             inputs="16 held-out Plummer mixtures and the isothermal sphere, n = 256")
        net.close()
    t = L.warm_start_trajectory(w, steps=10, Ks=(2,))
    last = {k: v[-1] for k, v in t["err_box_region"].items()}
    res["warm_start"] = {"steps": t["steps"], "err_box_region_last_step": last, "step_ms": t["step_ms"]}
    return res


def solver_vs_poisson(w, reps=5):
    """The AQUAL solve (K iterations) against a plain Poisson solve of the
    same density on the same box (pm_newton_potential: rho -> phi_N), best of
    reps, outside the timed region.  The paper reports its solver at 15 to 42
    times a standard Poisson solver (42 against 2 FFTs)."""
    import torch
    from paper_2312_02968_amd import mondpm as M
    p = w["params"]
    N = p["n_pad"]
    ctx = M.pm_create(p, len(w["mass"]))
    rho = torch.empty(N ** 3, device="cuda")
    M.pm_deposit(ctx, torch.from_numpy(w["pos"]).cuda(), torch.from_numpy(w["mass"]).cuda(), rho)
    phi = torch.empty_like(rho)

    def best(fn):
        fn()
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            fn()
            torch.cuda.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
        return min(t)
    t_poisson = best(lambda: M.pm_newton_potential(ctx, rho, phi))
    t_solve = best(lambda: M.aqual_solve(ctx, rho, phi, want_info=False))
    ctx.close()
    return {"poisson_ms": round(t_poisson, 3), "aqual_ms": round(t_solve, 3), "iterations": p["iters"],
            "ratio": round(t_solve / t_poisson, 2),
            "paper": "15-42x a standard Poisson solver (Python with FFTW, Intel Core i7-9750H)"}


def cpu_full_step(w):
    """One complete FP64 oracle step of the workload (deposit, K-iteration
    solve, kick and drift), each phase timed; with ORACLE_FFT_WORKERS set
    before the oracle is imported, the number of FFT threads.  Checks the
    extrapolation of cpu_baseline's bounded sample."""
    import numpy as np
    from oracle import pm as orc
    p = orc.Params.from_dict(w["params"])
    pos = w["pos"].astype(np.float64)
    vel = w["vel"].astype(np.float64)
    mass = w["mass"].astype(np.float64)
    dt = float(w["dt"])
    out = {"workload": w["workload"], "workers": orc.WORKERS, "cpu": host_cpu_model()}
    t0 = time.perf_counter()
    rho = orc.deposit(p, pos, mass)
    out["deposit_s"] = round(time.perf_counter() - t0, 2)
    print(f"cpu full step: deposit {out['deposit_s']} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    phi, _ = orc.aqual_solve(p, rho)
    out["solve_s"] = round(time.perf_counter() - t0, 2)
    del rho
    print(f"cpu full step: solve ({p.iters} iterations) {out['solve_s']} s", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    orc.interp_push(p, phi, pos, vel, dt, dt)
    out["gather_push_s"] = round(time.perf_counter() - t0, 2)
    out["step_s"] = round(out["deposit_s"] + out["solve_s"] + out["gather_push_s"], 2)
    out["steps_per_s"] = 1.0 / out["step_s"]
    return out


def increment_bytes(N, K, half):
    """Algorithmic HBM bytes of one increment solve (aqual_solve_increment,
    fixed K, no residual) by the same counting as pass_bytes: complex entries
    of 4 bytes (FP16 spectra) or 8 (FP32); the Newton spectrum of d_rho and
    the last one-component spectrum stay FP32; the linearised x passes also
    read the base field (3 R1)."""
    C1 = N * N * (N // 2 + 1)
    e = 4 if half else 8
    Ch, Cf = C1 * e, C1 * 8
    R1 = N ** 3 * 4
    b = R1 + Cf                       # x_fwd_real of d_rho
    b += 2 * Cf                       # y_fwd, one component, FP32
    b += Cf + Cf + 3 * Ch             # z_newton: rho_hat in, phi_N_hat and dg_N out
    b += 6 * Ch                       # y_inv
    b += K * (6 * Ch + 3 * R1)        # x(linearised nu)
    b += K * 6 * Ch                   # y_fwd
    b += (K - 1) * (6 * Ch + 6 * Ch + 6 * Ch + 3 * R1 + 6 * Ch + 6 * Ch + Cf + 6 * Ch)  # z, y, x(mu), y, z(div), y
    b += 3 * Ch + Cf                  # z_curl_final
    b += 2 * Cf + Cf + R1             # y_inv (one component) and x_inv_real
    return b


def incremental_record(w, K=2, reps=10):
    """The linearised increment solve (Sect. 5, item (v)) of one drift of the
    workload, about the fields of a 6-iteration solve of the starting density,
    outside the timed region: time per solve with FP32 and FP16 spectra
    (best of reps), algorithmic bytes, and the FP16 result against the FP32
    one."""
    import torch
    from paper_2312_02968_amd import mondpm as M
    p = w["params"]
    N = p["n_pad"]
    R = N ** 3
    ctx = M.pm_create(dict(p, iters=6, flags=p.get("flags", 0) | M.PM_F_RESIDUAL), len(w["mass"]))
    pos = torch.from_numpy(w["pos"]).cuda()
    vel = torch.from_numpy(w["vel"]).cuda()
    mass = torch.from_numpy(w["mass"]).cuda()
    rho = torch.empty(R, device="cuda")
    M.pm_deposit(ctx, pos, mass, rho)
    phi = torch.empty_like(rho)
    F = torch.empty(3 * R, device="cuda")
    M.aqual_solve_field(ctx, rho, phi, F, want_info=False)
    gM = torch.empty_like(F)
    M.pm_potential_field(ctx, phi, gM)
    rho1 = torch.empty_like(rho)
    M.pm_deposit(ctx, pos + float(w["dt"]) * vel, mass, rho1)
    drho = rho1 - rho
    del rho1
    ctx.close()
    ctx = M.pm_create(dict(p, iters=K), 0)
    out = {"K": K, "base_iterations": 6, "drift": "one step of the workload's dt"}
    res = {}
    for name, st in (("fp32", M.PM_STORE_FP32), ("fp16", M.PM_STORE_FP16)):
        d = torch.empty_like(rho)
        M.aqual_solve_increment(ctx, drho, F, gM, d, storage=st, want_info=False)
        torch.cuda.synchronize()
        t = []
        for _ in range(reps):
            t0 = time.perf_counter()
            M.aqual_solve_increment(ctx, drho, F, gM, d, storage=st, want_info=False)
            torch.cuda.synchronize()
            t.append((time.perf_counter() - t0) * 1e3)
        b = increment_bytes(N, K, st == M.PM_STORE_FP16)
        res[name] = d
        out[name] = {"ms": round(min(t), 3), "algorithmic_bytes": b,
                     "achieved_gbs": round(b / (min(t) * 1e-3) / 1e9, 1)}
    diff = (res["fp16"] - res["fp32"]).double().norm() / res["fp32"].double().norm()
    out["fp16_vs_fp32_dphi_rel_l2"] = float(f"{float(diff):.3e}")
    out["full_solve_bytes_K4"] = sum(v[0] for v in pass_bytes(N, p["iters"]).values())
    ctx.close()
    return out


def make_workload(name):
    import workloads as W
    if name == "isothermal":
        return W.isothermal_sphere(seed=0)
    if name == "ring":
        return W.ring(seed=0)
    if name == "two_body":
        return W.two_body()
    if name == "plummer512":
        return W.plummer_mixture(seed=0)
    raise SystemExit(f"unknown workload {name}")


def pass_bytes(N, K):
    """Algorithmic HBM bytes per step of each timed kernel kind, and launches per step.

    One complex spectrum component holds N * N * (N/2 + 1) valid entries of 8
    bytes (C1); a real grid holds N^3 floats (R1).  Each pass reads its input
    once and writes its output once.  The launch sequence is the one of one
    fixed-K solve: Newton (x, y, z, y), then per iteration x(nu), y, z(curl),
    y, x(mu), y, z(div), y, and in the last iteration x(nu), y, z(final).
    """
    C1 = N * N * (N // 2 + 1) * 8
    R1 = N ** 3 * 4
    b = {}
    b["x_fwd_real"] = (R1 + C1, 1)
    b["x_inv_real"] = (C1 + R1, 1)
    b["x_nu"] = (K * 6 * C1, K)
    b["x_mu"] = ((K - 1) * 6 * C1, K - 1)
    b["y_fwd"] = (2 * C1 + (2 * (K - 1) + 1) * 6 * C1, 2 * (K - 1) + 2)
    b["y_inv"] = (6 * C1 + 2 * (K - 1) * 6 * C1 + 2 * C1, 2 * (K - 1) + 2)
    b["z_newton"] = (C1 + C1 + 3 * C1, 1)
    b["z_curl"] = ((K - 1) * 6 * C1, K - 1)
    b["z_div"] = ((K - 1) * 7 * C1, K - 1)
    b["z_curl_final"] = (3 * C1 + C1, 1)
    b["fill"] = (R1, 1)
    return b


def oracle_error(w, n_sample=4096):
    """Force error of this configuration against the FP64 oracle on the same
    input, outside the timed region.

    The GPU deposits the workload's initial particles, runs the solve with the
    configuration's iterations and computes the smoothed force of every
    particle.  The oracle deposits all particles, solves the whole box and
    computes the force of n_sample of them.  Errors are relative to the
    sample's forces: L2, and the largest deviation over the largest force.
    """
    import numpy as np
    import torch
    from paper_2312_02968_amd import mondpm as M
    from oracle import pm as orc

    p = w["params"]
    n = len(w["mass"])
    R = p["n_pad"] ** 3
    ctx = M.pm_create(p, n)
    pos = torch.from_numpy(w["pos"]).cuda()
    mass = torch.from_numpy(w["mass"]).cuda()
    rho = torch.zeros(R, dtype=torch.float32, device="cuda")
    phi = torch.zeros(R, dtype=torch.float32, device="cuda")
    acc = torch.zeros(3 * n, dtype=torch.float32, device="cuda")
    M.pm_deposit(ctx, pos, mass, rho)
    M.aqual_solve(ctx, rho, phi, want_info=False)
    M.smooth_accel(ctx, phi, pos, acc)
    torch.cuda.synchronize()
    got = acc.cpu().numpy().reshape(-1, 3).astype(np.float64)
    ctx.close()
    del pos, mass, rho, phi, acc
    idx = np.random.default_rng(3).choice(n, n_sample, replace=False)
    op = orc.Params.from_dict(p)
    print(f"oracle error: FP64 deposit of {n} particles and solve of the {p['n_pad']}^3 box",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    rho_o = orc.deposit(op, w["pos"].astype(np.float64), w["mass"].astype(np.float64))
    phi_o, _ = orc.aqual_solve(op, rho_o)
    del rho_o
    ref = orc.smooth_accel(op, phi_o, w["pos"][idx].astype(np.float64))
    t = time.perf_counter() - t0
    d = got[idx] - ref
    return {"force_rel_l2": float(np.linalg.norm(d) / np.linalg.norm(ref)),
            "force_rel_max": float(np.abs(d).max() / np.abs(ref).max()),
            "sample": (f"deposit, {op.iters}-iteration solve and smoothed force from the initial state; "
                       f"forces of {n_sample} of {n} particles (seed 3) against the FP64 oracle"),
            "oracle_s": round(t, 1)}


def host_cpu_model():
    """The host CPU's model name from /proc/cpuinfo (None where it is not there)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(w, n_sample=4096):
    """FP64 oracle on a bounded sample of the workload, scaled to one step.

    Sample: the oracle's deposit and its gather + push on n_sample and on
    2 n_sample of the particles (a fixed part and a per-particle slope are
    fitted from the two and evaluated at N), its Newton solve on the full
    FFT box, and one full AQUAL iteration on the full box (nu, 3 FFTs,
    curl-free projection, 3 inverse FFTs, mu, 3 FFTs, divergence-free
    projection, 3 inverse FFTs).  A K-iteration step is the deposit, the
    Newton solve, K - 1 full iterations, a last one of nu, 3 FFTs, the
    projection and the inverse FFT of phi (timed as well), and the gather.
    """
    import numpy as np
    from oracle import pm as orc
    p = orc.Params.from_dict(w["params"])
    N = len(w["mass"])
    pos = w["pos"].astype(np.float64)
    mass = w["mass"].astype(np.float64)
    vel = w["vel"].astype(np.float64)
    idx = np.random.default_rng(0).choice(N, 2 * n_sample, replace=False)

    def timed(f):
        t0 = time.perf_counter()
        r = f()
        return time.perf_counter() - t0, r

    def fit(t1, t2):
        slope = max(t2 - t1, 0.0) / n_sample
        return max(t1 - slope * n_sample, 0.0) + slope * N

    d1, _ = timed(lambda: orc.deposit(p, pos[idx[:n_sample]], mass[idx[:n_sample]]))
    d2, rho = timed(lambda: orc.deposit(p, pos[idx], mass[idx] * (N / (2 * n_sample))))
    t_dep = fit(d1, d2)
    print(f"cpu baseline: deposit samples {d1:.1f} s, {d2:.1f} s", file=sys.stderr, flush=True)
    t_newton, (_, gN) = timed(lambda: orc.newton_potential(p, rho))
    print(f"cpu baseline: Newton solve {t_newton:.1f} s", file=sys.stderr, flush=True)
    del rho
    t0 = time.perf_counter()
    gM = orc.apply_nu(p, gN)
    gh, phih = orc.project_curl_free(p, np.stack([orc.fft3(gM[c]) for c in range(3)]))
    t_last_a = time.perf_counter() - t0
    t_last_b, phi = timed(lambda: orc.ifft3_real(phih))
    print(f"cpu baseline: nu, transforms and curl-free projection {t_last_a + t_last_b:.1f} s", file=sys.stderr,
          flush=True)
    t0 = time.perf_counter()
    gM = np.stack([orc.ifft3_real(gh[c]) for c in range(3)])
    del gh
    Fp = orc.apply_mu(p, gM)
    del gM
    Hh = orc.project_div_free(p, np.stack([orc.fft3((Fp - gN)[c]) for c in range(3)]))
    del Fp
    H = np.stack([orc.ifft3_real(Hh[c]) for c in range(3)])
    del Hh
    F = gN + H
    t_rest = time.perf_counter() - t0
    print(f"cpu baseline: rest of the iteration {t_rest:.1f} s", file=sys.stderr, flush=True)
    del H, F, gN
    g1, _ = timed(lambda: orc.interp_push(p, phi, pos[idx[:n_sample]], vel[idx[:n_sample]], 0.1, 0.1))
    g2, _ = timed(lambda: orc.interp_push(p, phi, pos[idx], vel[idx], 0.1, 0.1))
    t_gat = fit(g1, g2)
    K = p.iters
    t_iter = t_last_a + t_rest
    t_step = t_dep + t_gat + t_newton + (K - 1) * t_iter + t_last_a + t_last_b
    cores = orc.WORKERS
    return {"value": 1.0 / t_step, "unit": "PM steps/s", "cores": cores, "kind": "oracle",
            "cpu": host_cpu_model(),
            "sample": (f"FP64 oracle (scipy.fft, {cores} workers): deposit and gather+push of "
                       f"{n_sample} and {2 * n_sample} of {N} particles (fixed + per-particle cost "
                       f"fitted, evaluated at N), Newton solve and one full AQUAL iteration on the "
                       f"full {p.n_pad}^3 box; step = deposit + Newton + {K - 1} iterations + last "
                       f"iteration + gather; measured s: deposit {t_dep:.1f}, gather {t_gat:.1f}, "
                       f"newton {t_newton:.1f}, iteration {t_iter:.1f}, step {t_step:.1f}")}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="isothermal")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--timing", action="store_true", help="print per-kernel timing table to stderr")
    ap.add_argument("--copy-probe", action="store_true", help="only run the counter-calibration copy")
    ap.add_argument("--ingest-counters", metavar="DIR",
                    help="only write the counter summary from the rocprofv3 --pmc runs under DIR")
    ap.add_argument("--source-hash", help="with --ingest-counters: hash of the sources the runs were built from "
                                          "(default: the sources here)")
    ap.add_argument("--fft-compare", action="store_true",
                    help="only time this library's 512^3 real transforms beside rocFFT's")
    ap.add_argument("--warm", type=int, default=0, metavar="K",
                    help="time pm_step with the warm start (previous step's F) and K iterations")
    ap.add_argument("--no-starts", action="store_true",
                    help="skip the learned-start and warm-start comparisons")
    ap.add_argument("--no-oracle-error", action="store_true",
                    help="skip the force error against the FP64 oracle (about a minute of host work; "
                         "reported by default for FFT boxes up to 512^3 with the zero start)")
    ap.add_argument("--dft", choices=("fp32", "bf16x3"), default="fp32",
                    help="arithmetic of the y passes' radix-16 stage: FP32 butterflies (default) or "
                         "BF16x3 dense DFT-16 products on the matrix cores (PM_F_DFT_BF16X3)")
    ap.add_argument("--cpu-full", nargs="?", const="both", choices=("both", "sample"),
                    help="only time one complete FP64 oracle step of the workload and the bounded-sample "
                         "baseline ('sample': the baseline alone); no GPU; ORACLE_FFT_WORKERS sets the "
                         "FFT threads")
    ap.add_argument("--launch", choices=("graph", "eager"), default="graph",
                    help="time replays of the step recorded as a HIP graph (default) or eager pm_step calls")
    a = ap.parse_args()
    if a.copy_probe:
        copy_probe()
        return
    if a.ingest_counters:
        w = make_workload(a.workload)
        ingest_counters(a.ingest_counters, w["workload"], a.source_hash or source_hash(), w["params"]["iters"])
        return
    if a.fft_compare:
        fft_compare()
        return
    if a.cpu_full:
        w = make_workload(a.workload)
        rec = {"full_step": cpu_full_step(w)} if a.cpu_full == "both" else {}
        print("cpu baseline sample", file=sys.stderr, flush=True)
        rec["sample_baseline"] = cpu_baseline(w)
        print(json.dumps(rec), flush=True)
        return
    if a.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {a.gpus}); the path has no multi-GPU "
              "code, see the sharding note in the design document", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2312_02968_amd import mondpm as M

    w = make_workload(a.workload)
    if a.warm:
        w["params"] = dict(w["params"], iters=a.warm, flags=w["params"].get("flags", 0) | M.PM_F_WARM_START)
    if a.dft == "bf16x3":
        w["params"] = dict(w["params"], flags=w["params"].get("flags", 0) | M.PM_F_DFT_BF16X3)
    p = w["params"]
    N_part = len(w["mass"])
    dt = float(w["dt"])
    torch.cuda.init()
    stream = torch.cuda.Stream()
    ctx = M.pm_create(p, N_part, stream=stream)
    pos = torch.from_numpy(w["pos"]).cuda()
    vel = torch.from_numpy(w["vel"]).cuda()
    mass = torch.from_numpy(w["mass"]).cuda()
    torch.cuda.synchronize()
    for _ in range(a.warmup):
        M.pm_step(ctx, pos, vel, mass, dt)
    if a.warm and a.warmup == 0:
        M.pm_step(ctx, pos, vel, mass, dt)        # the warm start needs a previous solve
    torch.cuda.synchronize()
    ms_graph = None
    if a.launch == "graph":
        # The timed region: K replays of the whole step recorded as one HIP graph.
        M.pm_step_capture(ctx, pos, vel, mass, dt)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        M.pm_step_replay(ctx, a.steps)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        ms_graph = (t1 - t0) * 1e3 / a.steps
    # Eager steps with a HIP event pair around every launch on the library's
    # stream: the per-kernel durations of the roofline record (and the timed
    # region itself with --launch eager).
    M.pm_read_timing(ctx)
    M.pm_set_timing(ctx, True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(a.steps):
        M.pm_step(ctx, pos, vel, mass, dt)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = M.pm_read_timing(ctx)
    M.pm_set_timing(ctx, False)
    ms_eager = (t1 - t0) * 1e3 / a.steps
    ms_step = ms_graph if ms_graph is not None else ms_eager

    Npad = p["n_pad"]
    K = p["iters"]
    pb = pass_bytes(Npad, K)
    dom = max((k for k in timing if k in pb), key=lambda k: timing[k][0])
    tot_ms, launches = timing[dom]
    bytes_step, launches_step = pb[dom]
    avg_ms = tot_ms / launches
    bytes_launch = bytes_step / launches_step
    achieved = bytes_launch / (avg_ms * 1e-3) / 1e9
    if a.timing:
        for k, (t, c) in sorted(timing.items(), key=lambda kv: -kv[1][0]):
            extra = ""
            if k in pb:
                bb = pb[k][0] / pb[k][1]
                extra = f"  {bb / 1e9:.3f} GB/launch  {bb / (t / c * 1e-3) / 1e9:.0f} GB/s"
            print(f"{k:14s} {t / a.steps:8.3f} ms/step  {c // a.steps:3d} launches/step  "
                  f"{t / c:8.4f} ms/launch{extra}", file=sys.stderr)
    roof = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom, w["workload"]), "kernel": dom,
            "avg_launch_ms": round(avg_ms, 4), "algorithmic_bytes_per_launch": int(bytes_launch)}
    # particle kernels against the HBM roofline: algorithmic bytes 16 N + 4 n^3
    # (positions and masses read, the physical region of rho written) for the
    # deposit and 48 N + 4 n^3 (positions and velocities read and written, the
    # physical region of phi read) for the gather with kick and drift
    n_phys = p["n"]
    part = {}
    for k, b in (("deposit", 16 * N_part + 4 * n_phys ** 3), ("gather", 48 * N_part + 4 * n_phys ** 3),
                 ("sort", None)):
        if k in timing:
            t_ms = timing[k][0] / timing[k][1]
            part[k] = {"avg_launch_ms": round(t_ms, 4), "launches_per_step": timing[k][1] // a.steps}
            if b is not None:
                part[k].update(algorithmic_bytes=b, achieved_gbs=round(b / (t_ms * 1e-3) / 1e9, 1),
                               frac=round(b / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4))
    out = {
        "metric": METRIC,
        "value": round(1e3 / ms_step, 3),
        "unit": "PM steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["workload"], "grid": p["n"], "fft_box": Npad, "particles": N_part,
                   "iterations": K, "start": "warm" if a.warm else "zero", "sigma_cells": p["sigma"],
                   "mu": "standard" if p["mu"] == 0 else ("deep" if p["mu"] == 1 else "newton"), "dt": dt,
                   "dft": a.dft},
        "launch": a.launch,
        "ms_per_step_eager": round(ms_eager, 3),
        "particle_updates_per_s": round(N_part * 1e3 / ms_step, 1),
        "roofline": roof,
        "particle_kernels": part,
    }
    ctx.close()
    out["solver_vs_poisson"] = solver_vs_poisson(w)
    if not a.warm and a.dft == "fp32":
        out["incremental_step"] = incremental_record(w)
    if not a.no_starts and not a.warm and a.dft == "fp32":
        out.update(start_comparison(w))
    if not a.no_oracle_error and not a.warm and p["n_pad"] <= 512:
        out["oracle_error"] = oracle_error(w)
    if not a.no_cpu_baseline:
        print("cpu baseline: FP64 oracle on a bounded sample", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
