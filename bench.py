#!/usr/bin/env python3
"""Throughput of the decoupled phase-field step (Algorithm 1) on one MI355X.

Workload (the benchmark configuration of the 2D larger case): [0,1]^2, 20x20
spectral elements of order 8 (161 x 161 = 25,921 grid points per instance), a
sessile drop (half disc r = 0.25 at (0.5, 0), tanh profile eta = 0.01, contact
angle 90 deg), density ratio 1000, viscosity ratio 100, permittivity ratio 40,
closed box, V = 0 at the bottom and V_top in {0, 0.5, 1, 2} at the top: the four
voltages run as four instances of one context, dt = 5e-5.  Inputs are
synthetic and seeded (synth module); no dataset is involved.

Metric: DOF-steps/s = (grid points x instances) x steps / wall time of the
step loop (HIP events on the library's stream, inputs resident in HBM).  The
FP32-refined path (FP32 fast-diagonalisation solves + FP64 residual iterative
refinement) is the reported value; the plain FP64 path is timed beside it.

One JSON line is printed.  Extra keys:
  roofline      the dominant kernel class of the reported path, from HIP events the
                library records on its own stream around every launch during a second
                run of the same steps (pfd_profile_enable / pfd_profile_read):
                  fast-diagonalisation GEMM passes: algorithmic flops per launch
                    = Ny*Nx*(Nx+Ny)*planes (mean of the four passes 2*Ny*Nx*K*planes),
                    against the dense MFMA peak of their precision;
                  residual: algorithmic bytes per launch = 24*planes*Ny*Nx (read b, x;
                    write r), against HBM bandwidth;
  cpu_baseline  the FP64 oracle (NumPy/SciPy) on a bounded sample of the same
                workload (one instance, some steps after its one-time LU set-up).
"""
import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth import (C2, C3, C4, C5, c2_param_dict, c3_param_dict, c3_phi0, c4_instances,  # noqa: E402
                   c4_param_dict, c5_electrodes, c5_param_dict, c5_samples, c5_vd, drop_field)

VTOP = (0.0, 0.5, 1.0, 2.0)


def make_context_c3(precision, refine_max):
    """3D workload: 16x16 elements, K = 8, 128 Fourier planes, perturbed sphere."""
    import paper_2305_09020_amd as pfd
    xb = np.linspace(0.0, 1.0, C3["nx"] + 1)
    prob = pfd.make_problem(xb, xb, C3["K"], c3_param_dict(), [pfd.WALL] * 4, [1, 1, 0, 0],
                            nz=C3["nz"], lz=C3["lz"], precision=precision, refine_max=refine_max)
    ctx = pfd.Context(prob)
    x, y, z = ctx.coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    ctx.set_field("phi", c3_phi0(X, Y, Z))
    ctx.set_source("Vd", np.where(np.isclose(Y, 1.0), 1.0, 0.0))
    its = ctx.init_potential(tol=1e-12, max_iter=20000)
    return ctx, its


def make_context(precision, refine_max, workload="c2"):
    import paper_2305_09020_amd as pfd
    if workload == "c3":
        return make_context_c3(precision, refine_max)
    xb = np.linspace(0.0, 1.0, C2["nx"] + 1)
    prob = pfd.make_problem(xb, xb, C2["K"], c2_param_dict(), [pfd.WALL] * 4, [1, 1, 0, 0],
                            nbatch=len(VTOP), precision=precision, refine_max=refine_max)
    ctx = pfd.Context(prob)
    x, y, _ = ctx.coords()
    X, Y = np.meshgrid(x, y)
    phi = drop_field(X, Y, C2["center"], C2["r"], c2_param_dict()["eta"])
    ctx.set_field("phi", np.stack([phi] * len(VTOP)))
    vd = np.stack([np.where(np.isclose(Y, 1.0), v, 0.0) for v in VTOP])
    ctx.set_source("Vd", vd)
    its = ctx.init_potential(tol=1e-12, max_iter=20000)
    return ctx, its


class C4Run:
    """The batched workload: 64 independent 2D instances (n x n elements, n in 8..24, order
    4..10, seeded) on one stream, stepped through one hipGraph launch per step."""

    def __init__(self, precision, refine_max):
        import torch
        import paper_2305_09020_amd as pfd
        self.ctxs = []
        self.stream = torch.cuda.current_stream()
        for inst in c4_instances():
            xb = np.linspace(0.0, 1.0, inst["n"] + 1)
            par = c4_param_dict(inst["eps_ratio"])
            prob = pfd.make_problem(xb, xb, inst["K"], par, [pfd.WALL] * 4, [1, 1, 0, 0],
                                    precision=precision, refine_max=refine_max)
            ctx = pfd.Context(prob, stream=self.stream)
            x, y, _ = ctx.coords()
            X, Y = np.meshgrid(x, y)
            ctx.set_field("phi", drop_field(X, Y, C4["center"], C4["r"], par["eta"])[None])
            ctx.set_source("Vd", np.where(np.isclose(Y, 1.0), inst["vtop"], 0.0)[None])
            ctx.init_potential(tol=1e-12, max_iter=20000)
            self.ctxs.append(ctx)
        self.batch = pfd.Batch(self.ctxs, nlanes=4)
        self.dof = sum(c.planes * c.Nx * c.Ny for c in self.ctxs)

    def step(self, n):
        self.batch.step(n)

    step_async = step

    def diag(self):
        return dict(nonfinite=max(c.diag()["nonfinite"] for c in self.ctxs))


def roofline_c4(run, steps):
    """Dominant class over all instances: per-instance launch counts from an instrumented run
    (instances stepped by plain launches), per-instance average launch time from back-to-back
    replays; achieved = sum(launches x algorithmic flops or bytes) / sum(launches x time)."""
    for c in run.ctxs:
        c.profile_enable(True)
    run.batch.step(steps)
    profs = [c.profile_read() for c in run.ctxs]
    for c in run.ctxs:
        c.profile_enable(False)
    tot = {}
    for p in profs:
        for k, (ms, n) in p.items():
            if n > 0:
                a = tot.setdefault(k, [0.0, 0])
                a[0] += ms
                a[1] += n
    dom = max((k for k in tot if k in PEAK), key=lambda k: tot[k][0])
    work = 0.0
    time_s = 0.0
    for c, p in zip(run.ctxs, profs):
        n = p.get(dom, (0.0, 0))[1]
        if n == 0:
            continue
        avg = c.profile_replay(dom, 50) * 1e-6
        P, Nx, Ny = c.planes, c.Nx, c.Ny
        if dom.startswith("gemm"):
            per = float(Ny * Nx * (Nx + Ny) * P) * {0: 1.0, 1: 2.0, 2: 4.0 / 3.0}[c.solver_variant()[0]]
        else:
            per = float(24 * P * Nx * Ny)
        work += n * per
        time_s += n * avg
    scale = 1e12 if dom.startswith("gemm") else 1e9
    achieved = work / time_s / scale
    peak = PEAK[dom][0] / scale
    share = {k: round(v[0] / sum(x[0] for x in tot.values()), 4) for k, v in tot.items()}
    return {"bound": PEAK[dom][2], "achieved": achieved, "peak": peak, "unit": PEAK[dom][1],
            "frac": achieved / peak, "traffic": None, "kernel": dom,
            "avg_launch_us": time_s / max(1, sum(p.get(dom, (0, 0))[1] for p in profs)) * 1e6,
            "launches_per_step": tot[dom][1] / steps, "class_time_share": share,
            "note": "all 64 instances; per-launch work differs per instance"}


def cpu_baseline_c4(nsteps=10):
    """The FP64 oracle on the first instance of the batched workload, a few steps after its
    one-time sparse-LU factorisation."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
    from oracle.scheme import Scheme, Params, BCs, WALL
    inst = c4_instances()[0]
    par = Params(**c4_param_dict(inst["eps_ratio"]))
    xb = np.linspace(0.0, 1.0, inst["n"] + 1)
    m = Mesh2D(xb, xb, inst["K"])
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    sch = Scheme(m, par, bc)
    sch.set_state(drop_field(m.X, m.Y, C4["center"], C4["r"], par.eta).ravel())
    src = dict(Vd=np.where(np.isclose(m.Y.ravel(), 1.0), inst["vtop"], 0.0))
    sch.init_potential(src)
    t0 = time.perf_counter()
    sch.step(src)
    tset = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        sch.step(src)
    t = time.perf_counter() - t0
    return dict(value=m.Ng * nsteps / t, unit="DOF-steps/s", cores=1, kind="oracle",
                sample="instance 0 of the batch (%dx%d elements, K = %d), %d steps after the first; "
                       "first step incl. sparse-LU set-up %.1f s excluded; single-threaded SciPy/NumPy "
                       "(host has %d cores)" % (inst["n"], inst["n"], inst["K"], nsteps, tset,
                                                os.cpu_count() or 0))


def run_c5(a):
    """Equilibrium workload with the learned warm start: 12x12 elements of order 6 x 64
    Fourier planes, x-periodic, open top, bottom electrodes cycling (+V, gap, -V, gap); the
    equilibrium system (eq. 16, u = 0) marched to max|phi^{m+1} - phi^m| <= tol on one
    context whose permittivities and contact angle change per sample.  Training equilibria
    (seed 2) are generated by the march itself, the network is trained on the GPU by the
    library's kernels, and held-out problems (seed 3) are marched from the plain initial drop
    and from the network's mass-projected prediction."""
    import torch
    import paper_2305_09020_amd as pfd
    eta, dt, tol = C5["eta_run"], C5["dt_run"], C5["tol"]
    n_train = a.c5_train if a.c5_train is not None else C5["n_train_run"]
    n_test = a.c5_test if a.c5_test is not None else C5["n_test_run"]
    xb = np.linspace(0.0, C5["lx"], C5["nx"] + 1)
    yb = np.linspace(0.0, C5["ly"], C5["ny"] + 1)
    el = c5_electrodes()
    prob = pfd.make_problem(xb, yb, C5["K"], c5_param_dict(10.0, 90.0, dt=dt, eta=eta),
                            [pfd.WALL, pfd.OPEN, pfd.WALL, pfd.WALL], [0, 0, 0, 0], periodic_x=True,
                            nz=C5["nz"], lz=C5["lz"], precision=pfd.REFINED_FP32, refine_max=a.refine_max,
                            electrodes=[(x0, x1) for x0, x1, _ in el])
    ctx = pfd.Context(prob)
    ctx.set_graph(not a.no_graph)
    x, y, z = ctx.coords()
    Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
    phi0 = drop_field(X, Y, C5["center"][:2], C5["r"], eta, Z=Z, zc=C5["center"][2])
    wts = ctx.mass_weights()
    mass0 = float(np.sum(wts * phi0))
    N = phi0.size
    dof = N
    stats = dict(steps=0, seconds=0.0)

    zero = np.zeros(phi0.shape)

    def march(V, er, th, start):
        ctx.update_params(c5_param_dict(er, th, dt=dt, eta=eta))
        ctx.set_source("Vd", c5_vd(X, Y, V, el))
        for k in ("psi", "V"):           # no history from the previous problem
            ctx.set_field(k, zero)
            ctx.set_field(k, zero, level=-1)
        ctx.set_field("phi", start)
        ctx.init_potential(tol=1e-10, max_iter=5000)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        try:
            n, r = ctx.march_to_equilibrium(tol, C5["max_steps"])
            ok = True
        except pfd.PfdError as e:
            if e.code not in (pfd.ENOCONV, pfd.ENONFINITE):
                raise
            n, ok = C5["max_steps"] if e.code == pfd.ENOCONV else 0, False
        t = time.perf_counter() - t0
        stats["steps"] += n
        stats["seconds"] += t
        return n, t, ok

    t_gen = time.perf_counter()
    train = c5_samples(n_train, C5["seed_train"])
    T = torch.empty((n_train, N), dtype=torch.float32, device="cuda")
    kept = []
    for i, (V, er, th) in enumerate(train):
        n, t, ok = march(V, er, th, phi0)
        if ok:   # only equilibria the march reached to the tolerance become training data
            T[len(kept)] = torch.tensor(ctx.get_field("phi").ravel(), dtype=torch.float32, device="cuda")
            kept.append((V, er, th))
        print("# train %d/%d: %d steps %.2f s%s" % (i + 1, n_train, n, t, "" if ok else " (not converged)"),
              file=sys.stderr, flush=True)
    t_gen = time.perf_counter() - t_gen
    T = T[:len(kept)].contiguous()
    P = torch.tensor(np.stack([pfd.ws_inputs(*d) for d in kept]), device="cuda")
    ws = pfd.WarmStart(N, seed=C5["seed_train"])
    ws.init_output_bias(T)
    torch.cuda.synchronize()
    t_tr = time.perf_counter()
    hist = ws.train(P, T, steps=a.c5_train_steps, batch=32, lr=2e-3, seed=1)
    t_tr = time.perf_counter() - t_tr
    print("# trained %d steps in %.1f s: loss %.3g -> %.3g" % (a.c5_train_steps, t_tr, hist[0], hist[-1]),
          file=sys.stderr, flush=True)
    wt = torch.tensor(wts.ravel(), device="cuda")
    out = torch.empty(N, dtype=torch.float64, device="cuda")
    rows = []
    for i, (V, er, th) in enumerate(c5_samples(n_test, C5["seed_test"])):
        n_p, t_p, ok_p = march(V, er, th, phi0)
        e_p = ctx.stats()[0]["total"]
        f_p = ctx.get_field("phi").ravel()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ws.predict(pfd.ws_inputs(V, er, th), out, weights=wt, mass=mass0)
        torch.cuda.synchronize()
        t_pred = time.perf_counter() - t0
        start = out.cpu().numpy().reshape(phi0.shape)
        err0 = float(np.max(np.abs(start.ravel() - f_p)))
        n_w, t_w, ok_w = march(V, er, th, start)
        e_w = ctx.stats()[0]["total"]
        f_w = ctx.get_field("phi").ravel()
        rows.append(dict(steps_plain=n_p, steps_warm=n_w, converged_plain=ok_p, converged_warm=ok_w,
                         s_plain=t_p, s_warm=t_w + t_pred, energy_plain=e_p, energy_warm=e_w,
                         same_equilibrium=bool(abs(e_w - e_p) <= 1e-6 * abs(e_p)),
                         start_error=err0, energy_rel_diff=abs(e_w - e_p) / abs(e_p),
                         sorted_field_diff=float(np.max(np.abs(np.sort(f_w) - np.sort(f_p))))))
        print("# test %d: plain %d steps %.2f s, warm %d steps %.2f s (start error %.3g)"
              % (i, n_p, t_p, n_w, t_w + t_pred, err0), file=sys.stderr, flush=True)
    sp = np.array([r_["steps_plain"] for r_ in rows], dtype=float)
    sw = np.array([r_["steps_warm"] for r_ in rows], dtype=float)
    same = np.array([r_["same_equilibrium"] for r_ in rows])
    value = dof * stats["steps"] / stats["seconds"]
    out_line = {
        "metric": "DOF-steps/s on 1 GPU, FP32-refined vs plain FP64 at 1e-8 rel err; % roofline",
        "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": int(stats["steps"]), "warmup": 0,
        "ms_per_step": 1e3 * stats["seconds"] / stats["steps"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "config": {"workload": "3D equilibrium march with learned warm start: 12x12 elements order 6 x 64 "
                               "Fourier planes (336,384 points), x-periodic, open top, electrodes "
                               "(+V, gap, -V, gap) x 3, eta %g, dt %g, tol %g; V ~ U[0,2], eps ratio ~ "
                               "U[1.5,40], contact angle ~ U[60,120]; %d training / %d held-out problems"
                               % (eta, dt, tol, n_train, n_test),
                   "dof_per_step": dof, "graph": not a.no_graph, "refine_max": a.refine_max},
        "warm_start": {"train_samples": len(kept), "train_draws": n_train, "generation_s": t_gen, "train_steps": a.c5_train_steps,
                       "train_s": t_tr, "loss_first": float(hist[0]), "loss_last": float(np.mean(hist[-20:])),
                       "mean_steps_plain": float(sp.mean()), "mean_steps_warm": float(sw.mean()),
                       "step_ratio_plain_over_warm": float(sp.mean() / sw.mean()),
                       "same_equilibrium": int(same.sum()), "other_equilibrium": int((~same).sum()),
                       "step_ratio_same_equilibrium": float(sp[same].mean() / sw[same].mean()) if same.any() else None,
                       "other_equilibrium_lower_energy_warm": int(sum(1 for r_ in rows if not r_["same_equilibrium"]
                                                                       and r_["energy_warm"] < r_["energy_plain"])),
                       "mean_s_plain": float(np.mean([r_["s_plain"] for r_ in rows])),
                       "mean_s_warm": float(np.mean([r_["s_warm"] for r_ in rows])),
                       "max_energy_rel_diff": float(max(r_["energy_rel_diff"] for r_ in rows)),
                       "max_sorted_field_diff": float(max(r_["sorted_field_diff"] for r_ in rows)),
                       "per_problem": rows},
    }
    print(json.dumps(out_line), flush=True)


def time_steps(ctx, steps, warmup):
    import torch
    ctx.step(warmup)
    st = ctx.stream
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(st)
    ctx.step_async(steps)
    e1.record(st)
    torch.cuda.synchronize()
    d = ctx.diag()
    if d["nonfinite"]:
        raise RuntimeError("non-finite state during the timed steps")
    return e0.elapsed_time(e1) / 1e3


PEAK = {"gemm64": (78.6e12, "TFLOP/s", "mfma"), "gemm32": (157.3e12, "TFLOP/s", "mfma"),
        "residual": (8.0e12, "GB/s", "hbm")}


def roofline(ctx, steps, workload="c2", path="refined"):
    """Per-class kernel time over `steps` instrumented steps; roofline of the dominant
    class among those with an algorithmic per-launch figure."""
    ctx.profile_enable(True)
    ctx.step_async(steps)
    prof = ctx.profile_read()
    ctx.profile_enable(False)
    tot = {k: v for k, v in prof.items() if v[1] > 0}
    dom = max((k for k in tot if k in PEAK), key=lambda k: tot[k][0])
    ms, n = tot[dom]
    avg = ctx.profile_replay(dom, 200) * 1e-6     # back-to-back replay, no per-launch events
    avg_bracketed = ms / 1e3 / n
    P, Nx, Ny = ctx.planes, ctx.Nx, ctx.Ny
    variant, tune_us = ctx.solver_variant()
    if dom.startswith("gemm"):
        # four-pass variant: one GEMM pass per launch (mean 2*Ny*Nx*(Nx+Ny)/2 flops per plane);
        # fused strip variant: two passes per launch; fused middle passes: four in three
        per = float(Ny * Nx * (Nx + Ny) * P) * {0: 1.0, 1: 2.0, 2: 4.0 / 3.0}[variant]
        achieved = per / avg / 1e12
        peak = PEAK[dom][0] / 1e12
    else:
        per = float(24 * P * Nx * Ny)
        achieved = per / avg / 1e9
        peak = PEAK[dom][0] / 1e9
    share = {k: round(v[0] / sum(x[0] for x in tot.values()), 4) for k, v in tot.items()}
    return {"bound": PEAK[dom][2], "achieved": achieved, "peak": peak, "unit": PEAK[dom][1],
            "frac": achieved / peak, "traffic": traffic(dom, workload, path), "kernel": dom,
            "avg_launch_us": avg * 1e6, "avg_launch_us_event_bracketed": avg_bracketed * 1e6,
            "launches_per_step": n / steps, "per_launch": per, "class_time_share": share,
            "solver_variant": variant, "autotune_us_per_correction": tune_us,
            "residual_variant": ctx.residual_variant()[0], "autotune_us_residual": ctx.residual_variant()[1],
            "tuning": ctx.tuning(),
            "gemm_tile_config_per_site": ctx.gemm_config()[0]}


def traffic(dom, workload, path):
    """HBM bytes per launch of the class from the committed rocprofv3 counter summary
    profiles/hbm_traffic_<workload>.txt (FETCH_SIZE and WRITE_SIZE passes, scaled by a plain
    copy), only while pfd_kernels.hip is the source the counters were taken on; else None."""
    import hashlib
    f = os.path.join(ROOT, "profiles", "hbm_traffic_%s.txt" % workload)
    if not os.path.exists(f):
        return None
    src = os.path.join(ROOT, "paper_2305_09020_amd", "csrc", "pfd_kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    ok = False
    for line in open(f):
        if line.startswith("# kernel source sha256") and line.strip().endswith(sha):
            ok = True
        parts = line.split()
        if ok and len(parts) == 6 and parts[0] == path and parts[1] == dom:
            return float(parts[5])
    return None


def cpu_baseline(nsteps=40):
    """The FP64 oracle on one instance of the workload (V_top = 1): a few steps after
    its one-time sparse-LU factorisation (timed separately, not included)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
    from oracle.scheme import Scheme, Params, BCs, WALL
    par = Params(**c2_param_dict())
    xb = np.linspace(0.0, 1.0, C2["nx"] + 1)
    m = Mesh2D(xb, xb, C2["K"])
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    sch = Scheme(m, par, bc)
    sch.set_state(drop_field(m.X, m.Y, C2["center"], C2["r"], par.eta).ravel())
    src = dict(Vd=np.where(np.isclose(m.Y.ravel(), 1.0), 1.0, 0.0))
    sch.init_potential(src)
    t0 = time.perf_counter()
    sch.step(src)                      # first step factorises the constant matrices
    tset = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        sch.step(src)
    t = time.perf_counter() - t0
    return dict(value=m.Ng * nsteps / t, unit="DOF-steps/s", cores=1, kind="oracle",
                sample="one instance (V_top = 1) of the workload, %d steps after the first; "
                       "first step incl. sparse-LU set-up %.1f s excluded; SciPy SuperLU and "
                       "NumPy element loops run single-threaded (host has %d cores)"
                       % (nsteps, tset, os.cpu_count() or 0))


def cpu_baseline_c3(nsteps=1):
    """The FP64 oracle on the 3D workload at full size: one step after its first (the
    first includes the per-mode sparse-LU set-up, timed separately)."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
    from oracle.scheme import Scheme, Params, BCs, WALL
    par = Params(**c3_param_dict())
    xb = np.linspace(0.0, 1.0, C3["nx"] + 1)
    m = Mesh2D(xb, xb, C3["K"])
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    sch = Scheme(m, par, bc, Nz=C3["nz"], Lz=C3["lz"])
    Z = np.broadcast_to(sch.z[:, None], (C3["nz"], m.Ng))
    X = np.broadcast_to(m.X.ravel()[None, :], Z.shape)
    Y = np.broadcast_to(m.Y.ravel()[None, :], Z.shape)
    sch.set_state(c3_phi0(X, Y, Z))
    src = dict(Vd=np.where(np.isclose(Y, 1.0), 1.0, 0.0))
    sch.state["cur"]["V"] = np.array(Y)   # linear start V = y (the V0 fixed point is not timed)
    sch.state["old"]["V"] = sch.state["cur"]["V"].copy()
    t0 = time.perf_counter()
    sch.step(src)
    tset = time.perf_counter() - t0
    t0 = time.perf_counter()
    for _ in range(nsteps):
        sch.step(src)
    t = time.perf_counter() - t0
    dof = m.Ng * C3["nz"]
    return dict(value=dof * nsteps / t, unit="DOF-steps/s", cores=1, kind="oracle",
                sample="the 3D workload at full size, %d step(s) after the first; first step incl. "
                       "per-mode sparse-LU set-up %.1f s excluded; single-threaded SciPy/NumPy "
                       "(host has %d cores)" % (nsteps, tset, os.cpu_count() or 0))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["c2", "c3", "c4", "c5"], default="c2",
                    help="c2: the 2D benchmark configuration (default); c3: the 3D configuration; "
                         "c4: 64 uneven 2D instances in one batch; c5: equilibrium march with the "
                         "learned warm start (about 10 minutes)")
    ap.add_argument("--c5-train", type=int, default=None, help="training equilibria for c5")
    ap.add_argument("--c5-train-steps", type=int, default=3000)
    ap.add_argument("--c5-test", type=int, default=None, help="held-out problems for c5")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--refine-max", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the step kernels one by one instead of replaying a hipGraph")
    ap.add_argument("--only", choices=["refined", "fp64", "both"], default="both")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    a = ap.parse_args()
    if a.calibrate_copy:
        import torch
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 5 x %d bytes" % (src.numel() * 8))
        return
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the step would shard by Fourier mode in 3D; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2305_09020_amd as pfd
    torch.cuda.set_device(0)
    if a.workload == "c5":
        run_c5(a)
        return
    if a.steps is None:
        a.steps = {"c2": C2["steps"], "c3": C3["steps"], "c4": C4["steps"]}[a.workload]
    res = {}
    for name, prec in (("refined", pfd.REFINED_FP32), ("fp64", pfd.PLAIN_FP64)):
        if a.only not in (name, "both"):
            continue
        if a.workload == "c4":
            ctx, its = C4Run(prec, a.refine_max), 0
            t = time_steps(ctx, a.steps, a.warmup)
            dof = ctx.dof
            res[name] = dict(t=t, dof=dof, value=dof * a.steps / t, ctx=ctx,
                             roofline=roofline_c4(ctx, 5))
        else:
            ctx, its = make_context(prec, a.refine_max, a.workload)
            ctx.set_graph(not a.no_graph)
            t = time_steps(ctx, a.steps, a.warmup)
            dof = ctx.planes * ctx.Nx * ctx.Ny
            res[name] = dict(t=t, dof=dof, value=dof * a.steps / t, ctx=ctx,
                             roofline=roofline(ctx, min(a.steps, 200 if a.workload == "c2" else 20), a.workload, name))
        print("# %-7s %.3f ms/step  %.4e DOF-steps/s  (V0 fixed point: %d iterations)"
              % (name, 1e3 * t / a.steps, dof * a.steps / t, its), file=sys.stderr, flush=True)
    main_name = "refined" if "refined" in res else "fp64"
    r = res[main_name]
    out = {
        "metric": "DOF-steps/s on 1 GPU, FP32-refined vs plain FP64 at 1e-8 rel err; % roofline",
        "value": r["value"],
        "unit": "DOF-steps/s",
        "n_gpus": 1,
        "steps": a.steps,
        "warmup": a.warmup,
        "ms_per_step": 1e3 * r["t"] / a.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32" if main_name == "refined" else "f64",
        "data": "synthetic",
        "config": ({"workload": "2D sessile drop, 20x20 elements order 8 (25,921 points), "
                                "rho 1:1000, mu 1:100, eps 1:40, V_top {0,0.5,1,2} as 4 instances, "
                                "dt 5e-5, closed box; %s path" % main_name,
                    "instances": len(VTOP), "dof_per_step": r["dof"], "graph": not a.no_graph,
                    "refine_max": a.refine_max if main_name == "refined" else 0}
                   if a.workload == "c2" else
                   {"workload": "64 independent 2D drops in one batch (one hipGraph launch per step): "
                                "n x n elements with n ~ U{8..24}, order ~ U{4..10}, V_top ~ U[0,2], "
                                "eps ratio ~ U[1.5,40], seed 1, eta 0.02, dt 1e-4, closed boxes; "
                                "%s path" % main_name,
                    "instances": C4["n_inst"], "dof_per_step": r["dof"], "graph": True,
                    "refine_max": a.refine_max if main_name == "refined" else 0}
                   if a.workload == "c4" else
                   {"workload": "3D drop, 16x16 elements order 8 x 128 Fourier planes (Lz = 2, "
                                "2,130,048 points), perturbed sphere r = 0.3, rho 1:10, mu 1:2, "
                                "eps 1:10, dt 1e-4, walls; %s path" % main_name,
                    "instances": 1, "dof_per_step": r["dof"], "graph": not a.no_graph,
                    "refine_max": a.refine_max if main_name == "refined" else 0}),
    }
    out["roofline"] = r["roofline"]
    if "fp64" in res and "refined" in res:
        out["fp64_value"] = res["fp64"]["value"]
        out["refined_over_fp64"] = res["refined"]["value"] / res["fp64"]["value"]
        out["fp64_roofline"] = res["fp64"]["roofline"]
        if a.workload in ("c2", "c3"):
            # both contexts started from the same state and took the same steps (warmup,
            # timed, instrumented): field-wise max |refined - fp64| / max |fp64|
            n_cmp = a.warmup + a.steps + min(a.steps, 200 if a.workload == "c2" else 20)
            names = ("phi", "psi", "V", "P", "ux", "uy") + (("uz",) if a.workload == "c3" else ())
            errs = {}
            for k in names:
                f, g = res["fp64"]["ctx"].get_field(k), res["refined"]["ctx"].get_field(k)
                errs[k] = float(np.abs(g - f).max() / max(float(np.abs(f).max()), 1e-300))
            out["refined_vs_fp64"] = {"steps": n_cmp, "max_rel_err": errs}
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = {"c2": cpu_baseline, "c3": cpu_baseline_c3, "c4": cpu_baseline_c4}[a.workload]()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
