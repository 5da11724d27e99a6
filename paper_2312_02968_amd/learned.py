"""Training and evaluation of the learned starting guess, through the C ABI.

    python -m paper_2312_02968_amd.learned train [--pairs 256] [--epochs 40]
    python -m paper_2312_02968_amd.learned eval  [--weights PATH]

Training pairs come from the solver itself: random Plummer mixtures on a
128^3 region (256^3 FFT box) are deposited, the Newton potential gives the
network input, and a long solve (K iterations with its last F returned) gives
the target H = F - g_N.  Every step runs in the HIP library; this module only
draws the seeded particle sets, keeps the pairs in device tensors and orders
the calls.  The evaluation compares the learned start with the zero start on
held-out inputs: iterations and wall time to the accuracy of the plain K = 4
solve, and iterations in tolerance mode.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from paper_2312_02968_amd import mondpm as M  # noqa: E402
import workloads as W  # noqa: E402

WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "learned_start.npy")
# the same network at quarter resolution (voxels of 4^3 cells): cheaper to run
# and, trained the same way, the better start; the default of the comparison
WEIGHTS_Q4 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "learned_start_q4.npy")
DEFAULT_FACTOR = 4


def weights_for(factor):
    """The committed weights of the network at this block factor."""
    return WEIGHTS_Q4 if factor == 4 else WEIGHTS
TRAIN_N = 128
TARGET_ITERS = 12          # the long solve that defines the training target


def init_params(seed=0):
    """He-normal weights, zero biases, in the C ABI's parameter layout."""
    rng = np.random.default_rng(seed)
    shapes = [(4, 16, 3), (16, 16, 3), (16, 32, 3), (32, 32, 3), (32, 64, 3), (64, 64, 3),
              (96, 32, 3), (32, 32, 3), (48, 16, 3), (16, 16, 3), (16, 3, 1)]
    out = []
    for ci, co, k in shapes:
        taps = k ** 3
        std = np.sqrt(2.0 / (taps * ci)) * (0.1 if k == 1 else 1.0)
        out.append(rng.standard_normal(taps * ci * co) * std)
        out.append(np.zeros(co))
    v = np.concatenate(out).astype(np.float32)
    assert v.size == M.pm_net_param_count()
    return v


class PairMaker:
    """Builds (input, target) pairs for one region size on the GPU."""

    def __init__(self, n, max_particles, a0_ref=None):
        self.n = n
        self.N = 2 * n
        base = W.params(n, mu=W.MU_STANDARD, iters=TARGET_ITERS, flags=M.PM_F_RESIDUAL)
        self.base = base
        self.max_particles = max_particles
        self.ctx = None
        self.key = None

    def _ctx(self, p):
        key = (p["a0"], p["G"])
        if self.ctx is None or self.key != key:
            if self.ctx is not None:
                self.ctx.close()
            self.ctx = M.pm_create(p, self.max_particles)
            self.key = key
        return self.ctx

    def rho_of(self, ctx, w):
        rho = torch.empty(self.N ** 3, device="cuda")
        pos = torch.from_numpy(np.ascontiguousarray(w["pos"])).cuda()
        mass = torch.from_numpy(np.ascontiguousarray(w["mass"])).cuda()
        M.pm_deposit(ctx, pos, mass, rho)
        return rho

    def pair(self, net, slot, w):
        p = dict(self.base, a0=w["params"]["a0"], G=w["params"]["G"])
        ctx = self._ctx(p)
        rho = self.rho_of(ctx, w)
        phiN = torch.empty(self.N ** 3, device="cuda")
        M.pm_newton_potential(ctx, rho, phiN)
        M.pm_net_input(ctx, net, phiN, slot)
        phi = torch.empty(self.N ** 3, device="cuda")
        F = torch.empty(3 * self.N ** 3, device="cuda")
        info = M.aqual_solve_field(ctx, rho, phi, F)
        M.pm_net_target(ctx, net, phiN, F, slot)
        return info

    def close(self):
        if self.ctx is not None:
            self.ctx.close()
            self.ctx = None


def training_sample(seed, n=TRAIN_N):
    """Training mixture for an n^3 region; clump radii scale with n."""
    f = n / TRAIN_N
    return W.mixture_training_sample(seed, n=n, a_range=(2.0 * f, 8.0 * f))


def make_dataset(net, count, seed0=0, log=print, fb=2):
    """count pairs as device tensors X [count, 4 n^3] (BF16: the network reads
    its input in BF16, so nothing is lost) and Y [count, 3 n^3] (FP32), n the
    network size; the region is fb n / 2 cells per axis (its FFT box fb n).
    4096 pairs at n = 128 take 172 GB of device memory."""
    n = net.n
    region = fb * n // 2
    X = torch.empty(count, 4 * n ** 3, device="cuda", dtype=torch.bfloat16)
    Y = torch.empty(count, 3 * n ** 3, device="cuda")
    xin = torch.empty(4 * n ** 3, device="cuda")
    maker = PairMaker(region, 1 << 18)
    t0 = time.time()
    for i in range(count):
        w = training_sample(seed0 + i, region)
        maker.pair(net, 0, w)
        M.pm_net_get_input(net, 0, xin)
        X[i] = xin.to(torch.bfloat16)
        M.pm_net_get_target(net, 0, Y[i])
        if (i + 1) % 32 == 0 or i + 1 == count:
            torch.cuda.synchronize()
            log(f"pairs {i + 1}/{count}  {time.time() - t0:.1f} s")
    maker.close()
    return X, Y


def train(net, X, Y, epochs, batch=4, lr=3e-4, lr_final=None, seed=0, log=print):
    """Adam over shuffled mini-batches with a cosine learning-rate decay to
    lr_final (default lr / 10)."""
    if lr_final is None:
        lr_final = lr / 10.0
    rng = np.random.default_rng(seed)
    count = X.shape[0]
    steps_per_epoch = count // batch
    total = epochs * steps_per_epoch
    hist = []
    step = 0
    t0 = time.time()
    for ep in range(epochs):
        order = rng.permutation(count)
        acc = 0.0
        for s in range(steps_per_epoch):
            for b in range(batch):
                k = int(order[s * batch + b])
                M.pm_net_set_input(net, b, X[k].float() if X.dtype != torch.float32 else X[k])
                M.pm_net_set_target(net, b, Y[k])
            frac = step / max(total - 1, 1)
            cur = lr_final + 0.5 * (lr - lr_final) * (1.0 + np.cos(np.pi * frac))
            acc += M.pm_net_train_step(net, batch, float(cur))
            step += 1
        hist.append(acc / steps_per_epoch)
        log(f"epoch {ep + 1}/{epochs}  loss {hist[-1]:.4e}  {time.time() - t0:.1f} s")
    return hist


def save_params(path, v):
    os.makedirs(os.path.dirname(path), exist_ok=True)
    np.save(path, np.asarray(v, dtype=np.float32), allow_pickle=False)


def load_params(path=WEIGHTS):
    v = np.load(path, allow_pickle=False)
    if v.dtype != np.float32 or v.size != M.pm_net_param_count():
        raise ValueError(f"{path}: expected {M.pm_net_param_count()} float32 parameters")
    return v


# ---------------------------------------------------------------------------
# learned vs plain
# ---------------------------------------------------------------------------

def _timed(fn):
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    r = fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) * 1e3, r


def rejected(info):
    """The learned start is judged by its own solve: it is rejected when the
    tolerance solve from it did not converge or gave a non-finite residual, or
    when its second residual is not below its first (the start made the
    iteration worse instead of starting it closer to the fixed point)."""
    if info["status"] in (M.PM_E_NOTCONV, M.PM_E_NONFINITE):
        return True
    r = info["residuals"]
    return len(r) >= 2 and not (r[1] < r[0])


def learned_solve_tol(ctx, net, rho, phi):
    """The learned path in tolerance mode, with the plain iteration as the
    fallback: the solve from the learned start (aqual_solve_learned: features
    from the solve's own Newton spectrum, network, coarse start entering in
    Fourier space); if that solve is rejected, solve again from H = 0.
    Returns (info, fell_back); the time of both solves counts against the
    learned start."""
    info = M.aqual_solve_learned(ctx, net, rho, phi)
    if rejected(info):
        return M.aqual_solve(ctx, rho, phi), True
    return info, False


def compare_starts(w, net, K_plain=4, K_ref=30, tol=1e-4, max_iters=30, reps=3):
    """Learned vs zero start on one input (dict with params, pos, mass).

    Returns the potential error of the plain K_plain solve against a K_ref
    reference, the error of the learned start after K = 1..K_plain, the
    smallest K reaching the plain error, wall times (ms, best of reps) of the
    plain solve and of the learned path (Newton potential + network + solve
    with K iterations), and the iterations of both in tolerance mode."""
    p0 = dict(w["params"])
    n, N = p0["n"], p0["n_pad"]
    pos = torch.from_numpy(np.ascontiguousarray(w["pos"])).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(w["mass"])).cuda()
    out = {"workload": w.get("workload", ""), "n": n, "particles": int(pos.shape[0])}

    def ctx_for(**kw):
        return M.pm_create(dict(p0, **kw), pos.shape[0])

    c_ref = ctx_for(iters=K_ref)
    rho = torch.empty(N ** 3, device="cuda")
    M.pm_deposit(c_ref, pos, mass, rho)
    phi_ref = torch.empty_like(rho)
    M.aqual_solve(c_ref, rho, phi_ref)
    nref = float(torch.linalg.vector_norm(phi_ref))
    c_ref.close()

    phiN = torch.empty_like(rho)
    H0 = torch.empty(3 * N ** 3, device="cuda")
    phi = torch.empty_like(rho)
    c1 = ctx_for(iters=1)
    M.pm_newton_potential(c1, rho, phiN)
    M.pm_net_forward(c1, net, phiN, H0)

    def err(ph):
        return float(torch.linalg.vector_norm(ph - phi_ref)) / nref

    plain_err, learned_err = {}, {}
    for K in range(1, K_plain + 1):
        c = ctx_for(iters=K)
        M.aqual_solve(c, rho, phi)
        plain_err[K] = err(phi)
        M.aqual_solve(c, rho, phi, H0=H0)
        learned_err[K] = err(phi)
        c.close()
    target = plain_err[K_plain]
    K_star = next((K for K in range(1, K_plain + 1) if learned_err[K] <= target), None)
    out.update(plain_err=plain_err, learned_err=learned_err, K_plain=K_plain, K_learned=K_star)

    cp = ctx_for(iters=K_plain)
    t_plain = min(_timed(lambda: M.aqual_solve(cp, rho, phi, want_info=False))[0] for _ in range(reps))
    cp.close()
    if K_star is not None:
        # the learned path in one call; its start costs what it adds to a
        # plain solve with the same number of iterations
        cl = ctx_for(iters=K_star)
        t_learned = min(_timed(lambda: M.aqual_solve_learned(cl, net, rho, phi, want_info=False))[0]
                        for _ in range(reps))
        t_same = min(_timed(lambda: M.aqual_solve(cl, rho, phi, want_info=False))[0] for _ in range(reps))
        t_net = t_learned - t_same
        cl.close()
    else:
        t_learned = t_net = None
    out.update(t_plain_ms=t_plain, t_learned_ms=t_learned, t_start_ms=t_net)

    # tolerance mode: both starts iterate until r_k <= tol.  The fixed points
    # must agree.  The learned path is timed with its fallback: when the solve
    # from the learned start is rejected (see rejected()), the plain solve runs
    # as well, inside the timed path.
    ct = ctx_for(iters=max_iters, tol=tol)
    phi_l = torch.empty_like(rho)
    ip = M.aqual_solve(ct, rho, phi)
    il_raw = M.aqual_solve_learned(ct, net, rho, phi_l)
    il, fallback = learned_solve_tol(ct, net, rho, phi_l)
    fp_diff = float(torch.linalg.vector_norm(phi_l - phi)) / float(torch.linalg.vector_norm(phi))
    t_tol_plain = min(_timed(lambda: M.aqual_solve(ct, rho, phi, want_info=False))[0] for _ in range(reps))

    def learned_tol():
        learned_solve_tol(ct, net, rho, phi_l)
    t_tol_learned = min(_timed(learned_tol)[0] for _ in range(reps))
    ct.close()
    c1.close()
    out.update(tol=tol, tol_iters_plain=ip["iterations"],
               tol_iters_learned=il_raw["iterations"] + (il["iterations"] if fallback else 0),
               tol_status_plain=ip["status"], tol_status_learned=il["status"],
               tol_status_learned_start=il_raw["status"],
               resid_plain=ip["residuals"], resid_learned=il_raw["residuals"],
               tol_fixed_point_diff=fp_diff, tol_fallback=fallback,
               t_tol_plain_ms=t_tol_plain, t_tol_learned_ms=t_tol_learned)
    return out


def summarize(results):
    """Learned-vs-plain summary over inputs: median wall-time ratio in
    tolerance mode, largest fixed-point difference, fallback rate, and the
    iteration counts."""
    ratios = sorted(r["t_tol_learned_ms"] / r["t_tol_plain_ms"] for r in results)
    m = len(ratios)
    med = ratios[m // 2] if m % 2 else 0.5 * (ratios[m // 2 - 1] + ratios[m // 2])
    return {"inputs": m, "tol": results[0]["tol"], "median_time_ratio": med,
            "max_fixed_point_diff": max(r["tol_fixed_point_diff"] for r in results),
            "fallback_rate": sum(r["tol_fallback"] for r in results) / m,
            "iters_plain": [r["tol_iters_plain"] for r in results],
            "iters_learned": [r["tol_iters_learned"] for r in results]}


def warm_start_trajectory(w, steps=10, Ks=(2, 3), K_cold=4, K_ref=30, reps=5):
    """The paper's own start (Sect. 2.1): each solve begins from the previous
    step's field (PM_F_WARM_START).  A cold K_cold trajectory of pm_step moves
    the particles; along it, solves with the warm start and K iterations are
    compared with a cold K_ref reference at every step (potential error over
    the box and over the physical region), and pm_step is timed with each
    setting."""
    p0 = dict(w["params"])
    N, n = p0["n_pad"], p0["n"]
    lo = N // 2 - n // 2
    pos = torch.from_numpy(np.ascontiguousarray(w["pos"])).cuda()
    vel = torch.from_numpy(np.ascontiguousarray(w["vel"])).cuda()
    mass = torch.from_numpy(np.ascontiguousarray(w["mass"])).cuda()
    dt = float(w["dt"])
    Np = int(pos.shape[0])
    step_ctx = M.pm_create(dict(p0, iters=K_cold), Np)
    ref_ctx = M.pm_create(dict(p0, iters=K_ref), Np)
    cold_ctx = M.pm_create(dict(p0, iters=K_cold), Np)
    warm_ctx = {K: M.pm_create(dict(p0, iters=K, flags=M.PM_F_WARM_START), Np) for K in Ks}
    rho = torch.empty(N ** 3, device="cuda")
    phi_ref, phi = torch.empty_like(rho), torch.empty_like(rho)

    def errs(a, b):
        box = float(torch.linalg.vector_norm(a - b) / torch.linalg.vector_norm(b))
        a3, b3 = a.view(N, N, N)[lo:lo + n, lo:lo + n, lo:lo + n], b.view(N, N, N)[lo:lo + n, lo:lo + n, lo:lo + n]
        reg = float(torch.linalg.vector_norm(a3 - b3) / torch.linalg.vector_norm(b3))
        return box, reg

    hist = {"cold": [], **{f"warm{K}": [] for K in Ks}}
    for s in range(steps):
        M.pm_deposit(ref_ctx, pos, mass, rho)
        M.aqual_solve(ref_ctx, rho, phi_ref, want_info=False)
        M.aqual_solve(cold_ctx, rho, phi, want_info=False)
        hist["cold"].append(errs(phi, phi_ref))
        for K in Ks:
            M.aqual_solve(warm_ctx[K], rho, phi, want_info=False)
            hist[f"warm{K}"].append(errs(phi, phi_ref))
        M.pm_step(step_ctx, pos, vel, mass, dt, want_info=False)
    for c in (step_ctx, ref_ctx, cold_ctx, *warm_ctx.values()):
        c.close()

    # pm_step throughput, cold K_cold and warm K (fresh copies of the particles)
    timing = {}
    for name, K, flags in [("cold", K_cold, 0)] + [(f"warm{K}", K, M.PM_F_WARM_START) for K in Ks]:
        c = M.pm_create(dict(p0, iters=K, flags=flags), Np)
        pp, vv = pos.clone(), vel.clone()
        for _ in range(2):
            M.pm_step(c, pp, vv, mass, dt, want_info=False)
        ms = min(_timed(lambda: M.pm_step(c, pp, vv, mass, dt, want_info=False))[0] for _ in range(reps))
        timing[name] = ms
        c.close()
    return {"workload": w.get("workload", ""), "steps": steps, "dt": dt, "err_box_region": hist,
            "step_ms": timing}


def time_network(n, batch, reps=5, weights=None):
    """Forward and training-step times (ms, mean of reps after two warm-up
    calls) of the network at size n with random inputs and targets, and the
    rates against the forward pass's 115 872 flop per voxel (training: 3x)."""
    net = M.Net(n, batch)
    M.pm_net_set_params(net, load_params(weights) if weights else init_params(0))
    g = torch.Generator(device="cpu").manual_seed(0)
    for b in range(batch):
        M.pm_net_set_input(net, b, torch.randn(4 * n ** 3, generator=g).cuda())
        M.pm_net_set_target(net, b, 0.1 * torch.randn(3 * n ** 3, generator=g).cuda())

    def mean_ms(fn):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / reps

    fwd = mean_ms(lambda: M.pm_net_run(net, batch))
    trn = mean_ms(lambda: M.pm_net_train_step(net, batch, 1e-5, want_loss=False))
    net.close()
    flop = 115872.0 * n ** 3 * batch      # 54 cin cout per 3x3x3 layer over its level, 2 cin cout for the head
    return {"n": n, "batch": batch, "forward_ms": fwd, "train_step_ms": trn,
            "forward_tflops": flop / fwd * 1e-9, "train_tflops": 3 * flop / trn * 1e-9}


def held_out_inputs(n=256, count=4):
    """Held-out Plummer mixtures at n (radii twice the training range) and the
    isothermal sphere of the throughput workload."""
    f = n / TRAIN_N
    ws = [W.mixture_training_sample(100000 + i, n=n, a_range=(2.0 * f, 8.0 * f)) for i in range(count)]
    if n == 256:
        s = W.isothermal_sphere(seed=0)
        ws.append(dict(params=s["params"], pos=s["pos"], mass=s["mass"], workload=s.get("workload", "isothermal")))
    return ws


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("cmd", choices=["train", "eval", "warm", "time"])
    ap.add_argument("--pairs", type=int, default=256)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--batch", type=int, default=4)
    ap.add_argument("--lr", type=float, default=3e-4)
    ap.add_argument("--weights", default=None, help="network parameters (default: the committed ones for --factor)")
    ap.add_argument("--eval-n", type=int, default=256)
    ap.add_argument("--eval-count", type=int, default=16)
    ap.add_argument("--out", default=None, help="JSON file for the results")
    ap.add_argument("--train-n", type=int, default=TRAIN_N, help="region size (half the FFT box) for training")
    ap.add_argument("--factor", type=int, choices=(2, 4), default=DEFAULT_FACTOR,
                    help="box cells per network voxel along an axis (2: half resolution, 4: quarter)")
    ap.add_argument("--init", default=None, help="start training from these parameters")
    ap.add_argument("--seed0", type=int, default=0, help="first training seed")
    ap.add_argument("--tol", type=float, default=1e-4, help="eval: residual of the tolerance-mode comparison")
    a = ap.parse_args(argv)
    if a.weights is None:
        a.weights = weights_for(a.factor)
    log = lambda s: print(s, flush=True)  # noqa: E731
    torch.cuda.init()
    if a.cmd == "train":
        net = M.Net(2 * a.train_n // a.factor, a.batch)
        M.pm_net_set_params(net, load_params(a.init) if a.init else init_params(0))
        X, Y = make_dataset(net, a.pairs, seed0=a.seed0, log=log, fb=a.factor)
        hist = train(net, X, Y, a.epochs, batch=a.batch, lr=a.lr, log=log)
        save_params(a.weights, M.pm_net_get_params(net))
        res = {"pairs": a.pairs, "epochs": a.epochs, "n": a.train_n, "factor": a.factor, "loss": hist}
    elif a.cmd == "time":
        res = {"timings": [time_network(a.eval_n, 1), time_network(TRAIN_N, a.batch)]}
        log(json.dumps(res))
    elif a.cmd == "warm":
        res = warm_start_trajectory(W.isothermal_sphere(seed=0))
        log(json.dumps(res))
    else:
        v = load_params(a.weights)
        net = M.Net(2 * a.eval_n // a.factor, 1)
        M.pm_net_set_params(net, v)
        res = {"results": []}
        for w in held_out_inputs(a.eval_n, a.eval_count):
            r = compare_starts(w, net, tol=a.tol)
            log(json.dumps(r))
            res["results"].append(r)
        res["summary"] = summarize(res["results"])
        log(json.dumps({"summary": res["summary"]}))
    if a.out:
        with open(a.out, "w") as f:
            json.dump(res, f)
    return res


if __name__ == "__main__":
    main()
