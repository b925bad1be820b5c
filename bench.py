#!/usr/bin/env python3
"""Throughput of the decoupled phase-field step (Algorithms 1 and 2) on one MI355X.

Default workload (the 2D benchmark configuration): [0,1]^2, 20x20 spectral elements of
order 8 (161 x 161 = 25,921 grid points per instance), a sessile drop (half disc r = 0.25
at (0.5, 0), tanh profile eta = 0.01, contact angle 90 deg), density ratio 1000, viscosity
ratio 100, permittivity ratio 40, closed box, V = 0 at the bottom and V_top in
{0, 0.5, 1, 2} at the top as four instances of one context, dt = 5e-5.  Inputs are
synthetic and seeded (synth module); no dataset is involved.  Other workloads:
--workload c1 (4x4 elements, order 6), c3 (3D, 16x16 elements of order 8 x 128 Fourier
planes), c4 (64 uneven 2D instances in one batch), c5 (equilibrium march with the learned
warm start).

Metric: DOF-steps/s = (grid points x instances or planes) x steps / time of the step loop
(HIP events on the library's stream around the graph replays, inputs resident in HBM; the
median of three timed repeats).  The FP32-refined path (FP32 fast-diagonalisation
corrections + FP64 residual iterative refinement to its stop rule) is the reported value;
the plain FP64 path is timed beside it.

One JSON line is printed.  Extra keys:
  roofline      the whole step as one graph launch against HBM bandwidth: algorithmic bytes
                per step B_alg = F x 8 B x DOF with F the FP64 field passes the method needs
                (38 for the 2D full model, 46 for 3D, 16 for the equilibrium system), over the
                measured step time; traffic = HBM bytes per step from the rocprofv3
                FETCH_SIZE / WRITE_SIZE summary in profiles/ (while the kernel sources match
                it), plus the per-class split of the step (instrumented run).
  refinement    corrections per solve family and the last backward error of the refined path.
  cpu_baseline  the FP64 oracle (NumPy/SciPy) on a bounded sample of the same workload.
"""
import argparse
import json
import math
import os
import statistics
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

from synth import (C1, C2, C3, C4, C5, X6, c1_param_dict, c2_param_dict, c3_param_dict, c3_phi0,  # noqa: E402
                   c4_instances, c4_param_dict, c5_electrodes, c5_param_dict, c5_samples, c5_vd, drop_field,
                   x6_param_dict, x6_vd)

VTOP = (0.0, 0.5, 1.0, 2.0)
HBM_PEAK_GBS = 8000.0
MFMA_PEAK_TFLOPS = {"gemm32": 157.3, "gemm64": 78.6}   # MI355X dense FP32 / FP64 matrix peaks
FAMILIES = ("V", "psi", "phi", "P", "u")


class Run:
    """One benchmark workload on the GPU: a context (or a batch of contexts) on one stream."""

    def __init__(self, ctxs, dof, F, desc, batch=None, equilibrium=False):
        self.ctxs = ctxs
        self.ctx = ctxs[0]
        self.stream = self.ctx.stream
        self.dof = dof
        self.F = F
        self.desc = desc
        self.batch = batch
        self.equilibrium = equilibrium

    def step(self, n):
        if self.batch is not None:
            self.batch.step(n, self.equilibrium)
        else:
            self.ctx.step(n, self.equilibrium)

    def step_async(self, n):
        if self.batch is not None:
            self.batch.step(n, self.equilibrium)
        else:
            self.ctx.step_async(n, self.equilibrium)

    def nonfinite(self):
        return max(c.diag()["nonfinite"] for c in self.ctxs)


def _ctx2d(pfd, n, K, par, vtops, center, r, precision, stream=None):
    xb = np.linspace(0.0, 1.0, n + 1)
    prob = pfd.make_problem(xb, xb, K, par, [pfd.WALL] * 4, [1, 1, 0, 0], nbatch=len(vtops),
                            precision=precision)
    ctx = pfd.Context(prob, stream=stream)
    x, y, _ = ctx.coords()
    X, Y = np.meshgrid(x, y)
    phi = drop_field(X, Y, center, r, par["eta"])
    ctx.set_field("phi", np.stack([phi] * len(vtops)))
    ctx.set_source("Vd", np.stack([np.where(np.isclose(Y, 1.0), v, 0.0) for v in vtops]))
    ctx.init_potential(tol=1e-14, max_iter=20000)
    return ctx


def build_workload(name, precision, graph=True):
    """The GPU side of a workload (contexts built, initial potential solved)."""
    import torch
    import paper_2305_09020_amd as pfd
    if name == "c1":
        ctx = _ctx2d(pfd, C1["nx"], C1["K"], c1_param_dict(), C1["vtop"], C1["center"], C1["r"], precision)
        ctx.set_graph(graph)
        return Run([ctx], ctx.planes * ctx.Nx * ctx.Ny, 38,
                   "2D drop, 4x4 elements order 6 (625 points), rho 1:2, mu 1:2, eps 1:4, V_top 1, "
                   "dt 1e-4, closed box")
    if name == "c2":
        ctx = _ctx2d(pfd, C2["nx"], C2["K"], c2_param_dict(), VTOP, C2["center"], C2["r"], precision)
        ctx.set_graph(graph)
        return Run([ctx], ctx.planes * ctx.Nx * ctx.Ny, 38,
                   "2D sessile drop, 20x20 elements order 8 (25,921 points), rho 1:1000, mu 1:100, "
                   "eps 1:40, V_top {0,0.5,1,2} as 4 instances, dt 5e-5, closed box")
    if name == "c3":
        xb = np.linspace(0.0, 1.0, C3["nx"] + 1)
        prob = pfd.make_problem(xb, xb, C3["K"], c3_param_dict(), [pfd.WALL] * 4, [1, 1, 0, 0],
                                nz=C3["nz"], lz=C3["lz"], precision=precision)
        ctx = pfd.Context(prob)
        x, y, z = ctx.coords()
        Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
        ctx.set_field("phi", c3_phi0(X, Y, Z))
        ctx.set_source("Vd", np.where(np.isclose(Y, 1.0), 1.0, 0.0))
        ctx.init_potential(tol=1e-12, max_iter=20000)
        ctx.set_graph(graph)
        return Run([ctx], ctx.planes * ctx.Nx * ctx.Ny, 46,
                   "3D drop, 16x16 elements order 8 x 128 Fourier planes (Lz = 2, 2,130,048 points), "
                   "perturbed sphere r = 0.3, rho 1:10, mu 1:2, eps 1:10, dt 1e-4, walls")
    if name == "c4":
        stream = torch.cuda.current_stream()
        ctxs = []
        for i, inst in enumerate(c4_instances()):
            ctxs.append(_ctx2d(pfd, inst["n"], inst["K"], c4_param_dict(inst["eps_ratio"]), (inst["vtop"],),
                               C4["center"], C4["r"], precision, stream=stream))
            if (i + 1) % 16 == 0:
                print("# c4: %d instances created" % (i + 1), file=sys.stderr, flush=True)
        # one kernel configuration for every instance: the batch's multi-instance form merges the
        # k-th launches of instances that run the same kernel, so shared choices mean one launch
        # per step position.  The choice was measured on the merged launches (uniform
        # configurations swept, 20 steps each, one run): the four-pass solver with the
        # 2x2-tile, 4-slice split-K GEMM (configuration 7) on every pass and the per-node
        # residual with the order as a runtime argument (one kernel for all seven orders),
        # 2.02 ms per refined step (95 launches) against 2.34 with the LDS residual (one kernel
        # per order, 191 launches) and 2.65 with each instance's own autotuned choices;
        # configuration 2 (2x2 tiles, 2 slices) for the FP64 path, 1.19 against 1.26 ms.
        # Timings of this workload vary by a few percent between runs.
        if precision == pfd.REFINED_FP32:
            shared = [7] * 8 + [0, 0] + [0, 3, 1, 0, 0]
        else:
            shared = [2] * 8 + [0, 0] + [0, 1, 1, 0, 0]
        for c in ctxs:
            c.set_tuning(shared)
        batch = pfd.Batch(ctxs, nlanes=4)
        return Run(ctxs, sum(c.planes * c.Nx * c.Ny for c in ctxs), 38,
                   "64 independent 2D drops in one batch (multi-instance launches, one hipGraph launch "
                   "per step): n x n elements with n ~ U{8..24}, order ~ U{4..10}, V_top ~ U[0,2], eps "
                   "ratio ~ U[1.5,40], seed 1, eta 0.02, dt 1e-4, closed boxes", batch=batch)
    if name == "x6":
        par = x6_param_dict()
        xb = np.linspace(0.0, X6["lx"], X6["nx"] + 1)
        yb = np.linspace(0.0, X6["ly"], X6["ny"] + 1)
        prob = pfd.make_problem(xb, yb, X6["K"], par, [pfd.WALL, pfd.OPEN, pfd.WALL, pfd.WALL], [0, 0, 0, 0],
                                periodic_x=True, precision=precision,
                                electrodes=[(a, b) for a, b, _ in X6["electrodes"]])
        ctx = pfd.Context(prob)
        x, y, _ = ctx.coords()
        X, Y = np.meshgrid(x, y)
        ctx.set_field("phi", drop_field(X, Y, X6["center"], X6["r"], par["eta"])[None])
        ctx.set_source("Vd", x6_vd(X, Y)[None])
        ctx.init_potential(tol=1e-14, max_iter=20000)
        ctx.set_graph(graph)
        return Run([ctx], ctx.planes * ctx.Nx * ctx.Ny, 38,
                   "the paper's drop transport (Sec. 4.4.1): [0,1.6] x [0,0.5], 16x4 elements order 12 "
                   "(9,408 points), x-periodic, open top, electrodes -V,+V,-V,+V on the left half of the "
                   "bottom wall, semicircular drop r = 0.35 at (1.2, 0), Table 1 normalisation "
                   "(rho 235.9:235.9, mu 1:2, eps 1:8.1, eta 0.01, dt 1e-6)")
    if name in ("x3", "x4"):
        from synth import X3, X4, x3_param_dict, x3_electrodes, x4_mesh_y, x4_param_dict, x4_phi0, electrode_vd
        if name == "x3":
            el = x3_electrodes()
            prob = pfd.make_problem(np.linspace(0.0, X3["lx"], X3["nx"] + 1), np.array(X3["yb"]), X3["K"],
                                    x3_param_dict(), [pfd.WALL, pfd.OPEN, pfd.WALL, pfd.WALL], [0, 0, 0, 0],
                                    periodic_x=True, nz=X3["nz"], lz=X3["lz"], precision=precision,
                                    electrodes=[(a, b) for a, b, _ in el])
            ctx = pfd.Context(prob)
            x, y, z = ctx.coords()
            Z, Y, X = np.meshgrid(z, y, x, indexing="ij")
            ctx.set_field("phi", drop_field(X, Y, X3["center"][:2], X3["r"], X3["eta"], Z=Z, zc=X3["center"][2]))
            desc = ("the paper's 3D dielectric drop on an electrode array (Sec. 4.2), equilibrium system: "
                    "[0,5/3] x [0,2/3] x [0,3.5), 20x6 elements order 12 x 120 Fourier planes (2,102,400 "
                    "points), x-periodic, open top, ten electrodes alternating +-V0, hemisphere r = 0.5, "
                    "eps 1:32, eta 0.02, dt 2e-6")
        else:
            el = X4["electrodes"]
            prob = pfd.make_problem(np.linspace(0.0, X4["lx"], X4["nx"] + 1), x4_mesh_y(), X4["K"], x4_param_dict(),
                                    [pfd.WALL, pfd.OPEN, pfd.WALL, pfd.WALL], [0, 0, 0, 0], periodic_x=True,
                                    precision=precision, electrodes=[(a, b) for a, b, _ in el])
            ctx = pfd.Context(prob)
            x, y, _ = ctx.coords()
            X, Y = np.meshgrid(x, y)
            ctx.set_field("phi", x4_phi0(Y)[None])
            X, Y = X[None], Y[None]
            desc = ("the paper's dielectric film (Sec. 4.3), equilibrium system: [0,8] x [0,5], 16 x (5+4+4) "
                    "elements order 12 (30,144 points), x-periodic, open top, electrodes at 0 and V0, flat "
                    "film of thickness 1, eps 1:10, eta 0.01, S 2, dt 2e-6")
        ctx.set_source("Vd", electrode_vd(X, Y, el))
        ctx.init_potential(tol=1e-12, max_iter=20000)
        ctx.set_graph(graph)
        return Run([ctx], ctx.planes * ctx.Nx * ctx.Ny, 16, desc, equilibrium=True)
    raise ValueError("unknown workload %s" % name)


def time_steps(run, steps, warmup, repeats=3):
    """Seconds for `steps` steps: median of `repeats` timed loops (HIP events on the
    library's stream), after `warmup` untimed steps."""
    import torch
    run.step(warmup)
    st = run.stream
    ts = []
    for _ in range(repeats):
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(st)
        run.step_async(steps)
        e1.record(st)
        torch.cuda.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    if run.nonfinite():
        raise RuntimeError("non-finite state during the timed steps")
    return statistics.median(ts), ts


def probe_copy_bandwidth():
    """Device-to-device copy of 2 GiB (read + write 4 GiB moved): a measured HBM ceiling."""
    import torch
    a = torch.empty(2 ** 28, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(5):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    gbs = 5 * 2 * a.numel() * 8 / (e0.elapsed_time(e1) / 1e3) / 1e9
    del a, b
    return gbs


def probe_gemm_rate():
    """Dense square GEMMs through torch (hipBLASLt) in FP64 and FP32: a measured matrix-core
    ceiling for the fast-diagonalisation passes' classes (TFLOP/s)."""
    import torch
    out = {}
    for name, dt, n in (("fp64", torch.float64, 8192), ("fp32", torch.float32, 8192)):
        a = torch.randn(n, n, dtype=dt, device="cuda")
        b = torch.randn(n, n, dtype=dt, device="cuda")
        c = a @ b
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(5):
            c = a @ b
        e1.record()
        torch.cuda.synchronize()
        out[name] = round(5 * 2.0 * n ** 3 / (e0.elapsed_time(e1) / 1e3) / 1e12, 1)
        del a, b, c
    return out


def _sources_sha():
    import hashlib
    h = hashlib.sha256()
    cs = os.path.join(ROOT, "paper_2305_09020_amd", "csrc")
    for f in sorted(os.listdir(cs)):
        if f.endswith((".hip", ".cpp", ".h")):
            h.update(open(os.path.join(cs, f), "rb").read())
    return h.hexdigest()


def traffic(workload, path):
    """HBM bytes per step and per launch of each kernel class from the committed rocprofv3
    counter summary profiles/hbm_traffic_<workload>.txt (FETCH_SIZE and WRITE_SIZE passes over
    the steady-state steps, scaled by what the counters read for a plain device copy), only
    while the library sources hash to the value the counters were taken on; else None."""
    f = os.path.join(ROOT, "profiles", "hbm_traffic_%s.txt" % workload)
    if not os.path.exists(f):
        return None, {}
    sha = _sources_sha()
    ok = False
    step, per_class = None, {}
    for line in open(f):
        if line.startswith("# library sources sha256") and line.strip().endswith(sha):
            ok = True
        parts = line.split()
        if not ok or len(parts) < 3 or parts[1] != path:
            continue
        if parts[0] == "step":
            step = float(parts[2])
        elif parts[0] == "class" and len(parts) == 4:
            per_class[parts[2]] = float(parts[3])
    return step, per_class


def class_profile(run, steps):
    """Per kernel class: share of the step's kernel time, launches per step and the average
    launch (HIP events the library records around every launch during `steps` extra steps;
    the instrumented steps run eagerly)."""
    for c in run.ctxs:
        c.profile_enable(True)
    run.step(steps)
    tot = {}
    for c in run.ctxs:
        for k, (ms, n) in c.profile_read().items():
            if n:
                a = tot.setdefault(k, [0.0, 0])
                a[0] += ms
                a[1] += n
        c.profile_enable(False)
    all_ms = sum(v[0] for v in tot.values())
    return {k: {"share": round(v[0] / all_ms, 4), "launches_per_step": v[1] / steps,
                "avg_launch_us": round(1e3 * v[0] / v[1], 3)} for k, v in sorted(tot.items(), key=lambda kv: -kv[1][0])}


def roofline(run, t_step, workload, path, classes, probe_gbs):
    b_alg = float(run.F * 8 * run.dof)
    achieved = b_alg / t_step / 1e9
    step_traffic, class_traffic = traffic(workload, path)
    for k, v in (classes or {}).items():
        if k in class_traffic:
            v["traffic_per_launch"] = class_traffic[k]
            v["traffic_GBps"] = round(class_traffic[k] / (v["avg_launch_us"] * 1e-6) / 1e9, 1)
    out = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
           "traffic": step_traffic, "kernel": "whole step (one hipGraph launch)",
           "alg_bytes_per_step": b_alg, "field_passes_F": run.F, "dof": run.dof, "step_us": t_step * 1e6,
           "traffic_over_alg": (step_traffic / b_alg) if step_traffic else None,
           "probe_copy_GBps": probe_gbs, "frac_of_probe": achieved / probe_gbs if probe_gbs else None,
           "classes": classes}
    if run.batch is not None:
        out["kernel"] = "whole step (one hipGraph launch of multi-instance kernels)"
        out["launches_per_step"] = run.batch.launches()
        out["classes"] = "rocprofv3 kernel split: profiles/kernel_stats_%s.txt" % workload
    return out


def fdm_mfma(run, classes, refine, gemm_probe):
    """Matrix-core rate of the fast-diagonalisation passes, a kernel figure beside the step's
    HBM roofline: the dense flops of the corrections one step executes, 4 Ny Nx (Nx + Ny) per
    plane and correction (two passes along each axis), over the time per step of the GEMM
    classes (instrumented steps).  Corrections per family come from the refinement record of
    the last step (one per plane on the FP64 path and on the FP64 rung); where the residual
    kernel carries the first pass (residual variant 2) that pass's flops of every correction
    after a residual are left out, as its time is in the residual class.  The classes also hold
    the z transform's DFT GEMM of a plane count that is not a power of two (its flops are not
    counted).  None for batches."""
    if not classes or run.batch is not None:
        return None
    c = run.ctx
    Nx, Ny, planes = c.Nx, c.Ny, c.planes
    per = 4.0 * Ny * Nx * (Nx + Ny)
    p1 = 2.0 * Ny * Nx * Nx
    fams = ("V", "psi", "phi") if run.equilibrium else FAMILIES
    comps = {"u": 3 if c.planes_are_z else 2}
    fused = refine is not None and c.residual_variant()[0] == 2
    flops = {"gemm32": 0.0, "gemm64": 0.0}
    for f in fams:
        k = comps.get(f, 1)
        if refine is None:
            flops["gemm64"] += k * planes * per
            continue
        r = refine[f]
        n64 = r["fp64_planes"]
        corr = r["last_corrections"]
        flops["gemm64"] += k * n64 * per
        flops["gemm32"] += k * (planes - n64) * (corr * per - (max(corr - 1, 0) * p1 if fused else 0.0))
    out = {}
    for cls, fl in flops.items():
        v = classes.get(cls)
        if not fl or not v:
            continue
        us = v["avg_launch_us"] * v["launches_per_step"]
        tf = fl / (us * 1e-6) / 1e12
        probe = gemm_probe.get("fp32" if cls == "gemm32" else "fp64") if gemm_probe else None
        out[cls] = {"flops_per_step": fl, "us_per_step": round(us, 2), "achieved_TFLOPs": round(tf, 3),
                    "peak_TFLOPs": MFMA_PEAK_TFLOPS[cls], "frac": tf / MFMA_PEAK_TFLOPS[cls],
                    "frac_of_probe": tf / probe if probe else None}
    return out or None


def refinement(run):
    """Corrections per solve family of the last step and the most over the run (first
    context), FP64-rung planes, the last backward error and condition estimates."""
    st = run.ctx.refine_stats()
    return {f: {"fp64_planes": s["n_fp64_planes"], "last_corrections": s["last_corrections"],
                "max_corrections": s["max_corrections"], "failures": s["failures"],
                "last_eta": s["last_eta"], "kappa": [s["kappa_min"], s["kappa_max"]]}
            for f, s in zip(FAMILIES, st)}


# ------------------------------------------------------------------ the oracle on the host
def _oracle_run(workload):
    """(scheme, source dict, dof) of one oracle instance of the workload, initial state set."""
    from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
    from oracle.scheme import Scheme, Params, BCs, WALL
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    if workload in ("c1", "c2", "c4"):
        if workload == "c4":
            inst = c4_instances()[0]
            n, K, pd, v, cen, r = inst["n"], inst["K"], c4_param_dict(inst["eps_ratio"]), inst["vtop"], C4["center"], C4["r"]
        elif workload == "c2":
            n, K, pd, v, cen, r = C2["nx"], C2["K"], c2_param_dict(), 1.0, C2["center"], C2["r"]
        else:
            n, K, pd, v, cen, r = C1["nx"], C1["K"], c1_param_dict(), 1.0, C1["center"], C1["r"]
        par = Params(**pd)
        xb = np.linspace(0.0, 1.0, n + 1)
        m = Mesh2D(xb, xb, K)
        sch = Scheme(m, par, bc)
        sch.set_state(drop_field(m.X, m.Y, cen, r, par.eta).ravel())
        src = dict(Vd=np.where(np.isclose(m.Y.ravel(), 1.0), v, 0.0))
        sch.init_potential(src)
        return sch, src, m.Ng, "one instance (V_top = %g) of the workload, %dx%d elements, K = %d" % (v, n, n, K)
    if workload == "c5":
        from oracle.scheme import OPEN
        nz, eta = C5_ORACLE_PLANES, C5["eta_run"]
        par = Params(**c5_param_dict(10.0, 90.0, dt=C5["dt_run"], eta=eta))
        m = Mesh2D(np.linspace(0.0, C5["lx"], C5["nx"] + 1), np.linspace(0.0, C5["ly"], C5["ny"] + 1), C5["K"],
                   periodic_x=True)
        el = c5_electrodes()
        sch = Scheme(m, par, BCs(side={BOTTOM: WALL, TOP: OPEN}, electrodes=[(a, b_) for a, b_, _ in el]),
                     Nz=nz, Lz=C5["lz"])
        Z = np.broadcast_to(sch.z[:, None], (nz, m.Ng))
        X = np.broadcast_to(m.X.ravel()[None, :], Z.shape)
        Y = np.broadcast_to(m.Y.ravel()[None, :], Z.shape)
        sch.set_state(drop_field(X, Y, C5["center"][:2], C5["r"], eta, Z=Z, zc=C5["center"][2]))
        src = dict(Vd=c5_vd(X, Y, 1.0, el))
        sch.init_potential(src)
        return sch, src, m.Ng * nz, ("the equilibrium workload's mesh (12x12 elements, K = 6) with %d of its %d "
                                     "Fourier planes, equilibrium steps (V = 1, eps ratio 10, contact angle 90)"
                                     % (nz, C5["nz"]))
    if workload == "x6":
        from oracle.scheme import OPEN
        par = Params(**x6_param_dict())
        m = Mesh2D(np.linspace(0.0, X6["lx"], X6["nx"] + 1), np.linspace(0.0, X6["ly"], X6["ny"] + 1), X6["K"],
                   periodic_x=True)
        bcx = BCs(side={BOTTOM: WALL, TOP: OPEN}, electrodes=[(a, b) for a, b, _ in X6["electrodes"]])
        sch = Scheme(m, par, bcx)
        sch.set_state(drop_field(m.X, m.Y, X6["center"], X6["r"], par.eta).ravel())
        src = dict(Vd=x6_vd(m.X.ravel(), m.Y.ravel()))
        sch.init_potential(src)
        return sch, src, m.Ng, "the drop-transport workload at full size"
    par = Params(**c3_param_dict())
    xb = np.linspace(0.0, 1.0, C3["nx"] + 1)
    m = Mesh2D(xb, xb, C3["K"])
    nz = C3_ORACLE_PLANES    # a bounded sample: the oracle's cost is linear in the planes
    sch = Scheme(m, par, bc, Nz=nz, Lz=C3["lz"])
    Z = np.broadcast_to(sch.z[:, None], (nz, m.Ng))
    X = np.broadcast_to(m.X.ravel()[None, :], Z.shape)
    Y = np.broadcast_to(m.Y.ravel()[None, :], Z.shape)
    sch.set_state(c3_phi0(X, Y, Z))
    src = dict(Vd=np.where(np.isclose(Y, 1.0), 1.0, 0.0))
    sch.state["cur"]["V"] = np.array(Y)   # linear start V = y (the V0 fixed point is not timed)
    sch.state["old"]["V"] = sch.state["cur"]["V"].copy()
    return sch, src, m.Ng * nz, ("the 3D workload's mesh (16x16 elements, K = 8) with %d of its %d Fourier "
                                 "planes" % (nz, C3["nz"]))


C3_ORACLE_PLANES = 16
C5_ORACLE_PLANES = 8


def cpu_baseline(workload, nsteps, equilibrium=False):
    """The FP64 oracle (sparse LU, NumPy element loops) on the host: `nsteps` steps after its
    first (which includes the one-time LU factorisations, timed separately), once with the
    BLAS / OpenMP pools held to one thread and then `nsteps` more with all of them."""
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from threadpoolctl import threadpool_limits, threadpool_info
    res = {}
    sch, src, dof, what = _oracle_run(workload)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        sch.step(src, equilibrium=equilibrium)
        tset = time.perf_counter() - t0
    print("# oracle baseline: first step (with the sparse-LU set-up) %.1f s" % tset, file=sys.stderr, flush=True)
    for label, lim in (("one", 1), ("all", None)):
        with threadpool_limits(limits=lim):
            t0 = time.perf_counter()
            for i in range(nsteps):
                sch.step(src, equilibrium=equilibrium)
                if (i + 1) % 10 == 0 or i + 1 == nsteps:
                    print("# oracle baseline (%s): %d/%d steps, %.1f s" % (label, i + 1, nsteps,
                                                                          time.perf_counter() - t0),
                          file=sys.stderr, flush=True)
            res[label] = (dof * nsteps / (time.perf_counter() - t0), tset)
    threads = max([p.get("num_threads", 1) for p in threadpool_info()] + [1])
    return dict(value=res["one"][0], unit="DOF-steps/s", cores=1, kind="oracle",
                value_all_threads=res["all"][0], threads_all=threads,
                sample="%s, %d steps after the first (first step incl. sparse-LU set-up %.1f s excluded); "
                       "SciPy SuperLU (sequential) and NumPy; value: BLAS pools at one thread; "
                       "value_all_threads: %d further steps with the pools at %d threads; host has %d cores"
                       % (what, nsteps, tset, nsteps, threads, os.cpu_count() or 0))


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
                            nz=C5["nz"], lz=C5["lz"], precision=pfd.REFINED_FP32,
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

    def march(V, er, th, start, max_steps=C5["max_steps"]):
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
            n, r = ctx.march_to_equilibrium(tol, max_steps)
            ok = True
        except pfd.PfdError as e:
            if e.code not in (pfd.ENOCONV, pfd.ENONFINITE):
                raise
            n, ok = max_steps if e.code == pfd.ENOCONV else 0, False
        t = time.perf_counter() - t0
        stats["steps"] += n
        stats["seconds"] += t
        return n, t, ok

    t_gen = time.perf_counter()
    train = c5_samples(n_train, C5["seed_train"])
    T = torch.empty((n_train, N), dtype=torch.float32, device="cuda")
    kept = []
    for i, (V, er, th) in enumerate(train):
        n, t, ok = march(V, er, th, phi0, C5["gen_max_steps"])
        if ok:   # only equilibria the march reached to the tolerance become training data
            T[len(kept)] = torch.tensor(ctx.get_field("phi").ravel(), dtype=torch.float32, device="cuda")
            kept.append((V, er, th))
        print("# train %d/%d: %d steps %.2f s%s" % (i + 1, n_train, n, t, "" if ok else " (not converged)"),
              file=sys.stderr, flush=True)
    t_gen = time.perf_counter() - t_gen
    T = T[:len(kept)].contiguous()
    P = torch.tensor(np.stack([pfd.ws_inputs(*d) for d in kept]), device="cuda")
    ws = pfd.WarmStart(phi0.shape, periodic=(True, False, True), seed=C5["seed_train"])
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
        dmax = float(np.max(np.abs(f_w - f_p)))
        m_p, m_w = float(np.sum(wts.ravel() * f_p)), float(np.sum(wts.ravel() * f_w))
        rows.append(dict(steps_plain=n_p, steps_warm=n_w, converged_plain=ok_p, converged_warm=ok_w,
                         s_plain=t_p, s_warm=t_w + t_pred, energy_plain=e_p, energy_warm=e_w,
                         same_equilibrium=bool(ok_p and ok_w and dmax <= 1e-4),
                         start_error=err0, field_diff=dmax, mass_rel_diff=abs(m_w - m_p) / abs(m_p),
                         energy_rel_diff=abs(e_w - e_p) / abs(e_p),
                         sorted_field_diff=float(np.max(np.abs(np.sort(f_w) - np.sort(f_p))))))
        print("# test %d: plain %d steps %.2f s, warm %d steps %.2f s (start error %.3g, final |dphi| %.3g)"
              % (i, n_p, t_p, n_w, t_w + t_pred, err0, dmax), file=sys.stderr, flush=True)
    sp = np.array([r_["steps_plain"] for r_ in rows], dtype=float)
    sw = np.array([r_["steps_warm"] for r_ in rows], dtype=float)
    same = np.array([r_["same_equilibrium"] for r_ in rows])
    value = dof * stats["steps"] / stats["seconds"]
    out_line = {
        "metric": "DOF-steps/s on 1 GPU, FP32-refined vs plain FP64 at 1e-8 rel err; % roofline",
        "value": value, "unit": "DOF-steps/s", "n_gpus": 1, "steps": int(stats["steps"]), "warmup": 0,
        "ms_per_step": 1e3 * stats["seconds"] / stats["steps"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32", "data": "synthetic",
        "roofline": {"bound": "hbm", "achieved": 16 * 8 * dof * stats["steps"] / stats["seconds"] / 1e9,
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": 16 * 8 * dof * stats["steps"] / stats["seconds"] / 1e9 / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "whole equilibrium step (F = 16 field passes), host-synchronised march"},
        "config": {"workload": "3D equilibrium march with learned warm start: 12x12 elements order 6 x 64 "
                               "Fourier planes (336,384 points), x-periodic, open top, electrodes "
                               "(+V, gap, -V, gap) x 3, eta %g, dt %g, tol %g; V ~ U[0,2], eps ratio ~ "
                               "U[1.5,40], contact angle ~ U[60,120]; %d training / %d held-out problems"
                               % (eta, dt, tol, n_train, n_test),
                   "dof_per_step": dof, "graph": not a.no_graph},
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
                       "max_mass_rel_diff": float(max(r_["mass_rel_diff"] for r_ in rows)),
                       "max_field_diff_same": float(max([r_["field_diff"] for r_ in rows if r_["same_equilibrium"]]
                                                        or [float("nan")])),
                       "max_sorted_field_diff": float(max(r_["sorted_field_diff"] for r_ in rows)),
                       "per_problem": rows},
    }
    if not a.no_cpu_baseline:
        out_line["cpu_baseline"] = cpu_baseline("c5", 20, equilibrium=True)
    print(json.dumps(out_line), flush=True)




def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--workload", choices=["c1", "c2", "c3", "c4", "c5", "x6", "x3", "x4"], default="c2",
                    help="c2: the 2D benchmark configuration (default); c1: its small case; c3: the 3D "
                         "configuration; c4: 64 uneven 2D instances in one batch; c5: equilibrium march "
                         "with the learned warm start (about 10 minutes); x6: the paper's drop transport; x3, x4: "
                         "the paper's 3D drop and 2D film equilibrium marches")
    ap.add_argument("--c5-train", type=int, default=None, help="training equilibria for c5")
    ap.add_argument("--c5-train-steps", type=int, default=3000)
    ap.add_argument("--c5-test", type=int, default=None, help="held-out problems for c5")
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--repeats", type=int, default=3, help="timed loops; the median is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-graph", action="store_true",
                    help="launch the step kernels one by one instead of replaying a hipGraph")
    ap.add_argument("--only", choices=["refined", "fp64", "both"], default="both")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (reference for the "
                         "FETCH_SIZE / WRITE_SIZE counters) and exit")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this library has no multi-GPU path "
              "(the step would shard by Fourier mode in 3D; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2305_09020_amd as pfd
    if a.calibrate_copy:
        src = torch.ones(32 * 1024 * 1024, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print("copied 5 x %d bytes" % (src.numel() * 8))
        return
    torch.cuda.set_device(0)
    if a.workload == "c5":
        run_c5(a)
        return
    if a.steps is None:
        a.steps = {"c1": C1["steps"], "c2": C2["steps"], "c3": C3["steps"], "c4": C4["steps"],
                   "x6": X6["steps"], "x3": 200, "x4": 500}[a.workload]
    probe = probe_copy_bandwidth()
    gemm_probe = probe_gemm_rate()
    res = {}
    for name, prec in (("refined", pfd.REFINED_FP32), ("fp64", pfd.PLAIN_FP64)):
        if a.only not in (name, "both"):
            continue
        run = build_workload(a.workload, prec, graph=not a.no_graph)
        t, ts = time_steps(run, a.steps, a.warmup, a.repeats)
        nprof = min(a.steps, 50 if a.workload in ("c1", "c2", "x6", "x4") else 10)
        # the instrumented steps run eagerly, which for a batch would time each instance's own
        # launches rather than the multi-instance ones: a batch's per-kernel split is the
        # rocprofv3 summary of its graph replays instead
        classes = class_profile(run, nprof) if run.batch is None else None
        if run.batch is not None:
            nprof = 0
        refine = refinement(run) if prec == pfd.REFINED_FP32 else None
        rl = roofline(run, t / a.steps, a.workload, name, classes, probe)
        rl["fdm_mfma"] = fdm_mfma(run, classes, refine, gemm_probe)
        res[name] = dict(t=t, ts=ts, run=run, value=run.dof * a.steps / t,
                         roofline=rl, refinement=refine,
                         nsteps=a.warmup + a.repeats * a.steps + nprof)
        print("# %-7s %.3f ms/step  %.4e DOF-steps/s  (repeats: %s ms/step)"
              % (name, 1e3 * t / a.steps, run.dof * a.steps / t,
                 " ".join("%.3f" % (1e3 * x / a.steps) for x in ts)), file=sys.stderr, flush=True)
    main_name = "refined" if "refined" in res else "fp64"
    r = res[main_name]
    out = {
        "metric": "DOF-steps/s on 1 GPU, FP32-refined vs plain FP64 at 1e-8 rel err; % roofline",
        "value": r["value"], "unit": "DOF-steps/s", "n_gpus": 1, "steps": a.steps, "warmup": a.warmup,
        "ms_per_step": 1e3 * r["t"] / a.steps, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f64+f32" if main_name == "refined" else "f64", "data": "synthetic",
        "config": {"workload": r["run"].desc + "; %s path" % main_name, "dof_per_step": r["run"].dof,
                   "graph": not a.no_graph, "timed_repeats": a.repeats},
        "roofline": dict(r["roofline"], probe_gemm_TFLOPs=gemm_probe),
    }
    if r["refinement"]:
        out["refinement"] = r["refinement"]
    if "fp64" in res and "refined" in res:
        out["fp64_value"] = res["fp64"]["value"]
        out["fp64_ms_per_step"] = 1e3 * res["fp64"]["t"] / a.steps
        out["refined_over_fp64"] = res["refined"]["value"] / res["fp64"]["value"]
        out["fp64_roofline"] = res["fp64"]["roofline"]
        if a.workload not in ("c4",):
            # both contexts started from the same state and took the same steps (warm-up,
            # timed, instrumented): field-wise max |refined - fp64| / max |fp64|
            names = ((("phi", "psi", "V") if a.workload in ("x3", "x4") else ("phi", "psi", "V", "P", "ux", "uy"))
                     + (("uz",) if a.workload == "c3" else ()))
            errs = {}
            for k in names:
                f, g = res["fp64"]["run"].ctx.get_field(k), res["refined"]["run"].ctx.get_field(k)
                errs[k] = float(np.abs(g - f).max() / max(float(np.abs(f).max()), 1e-300))
            out["refined_vs_fp64"] = {"steps": res["refined"]["nsteps"], "max_rel_err": errs}
    if not a.no_cpu_baseline and a.workload not in ("x3", "x4"):
        out["cpu_baseline"] = cpu_baseline(a.workload, {"c1": 100, "c2": 40, "c3": 4, "c4": 10, "x6": 60}[a.workload])
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
