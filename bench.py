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
  roofline      dominant kernel (FP32 or FP64 fast-diagonalisation pass) against the
                vector-ALU peak of its precision, from per-kernel HIP-event timing
                done inside the library on its stream (pfd_time_kernel);
  cpu_baseline  the FP64 oracle (NumPy/SciPy) on a bounded sample of the same
                workload (one instance, a few steps after its one-time LU set-up).
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

from synth import C2, c2_param_dict, drop_field  # noqa: E402

VTOP = (0.0, 0.5, 1.0, 2.0)


def make_context(precision, refine_iters):
    import paper_2305_09020_amd as pfd
    xb = np.linspace(0.0, 1.0, C2["nx"] + 1)
    prob = pfd.make_problem(xb, xb, C2["K"], c2_param_dict(), [pfd.WALL] * 4, [1, 1, 0, 0],
                            nbatch=len(VTOP), precision=precision, refine_iters=refine_iters)
    ctx = pfd.Context(prob)
    x, y, _ = ctx.coords()
    X, Y = np.meshgrid(x, y)
    phi = drop_field(X, Y, C2["center"], C2["r"], c2_param_dict()["eta"])
    ctx.set_field("phi", np.stack([phi] * len(VTOP)))
    vd = np.stack([np.where(np.isclose(Y, 1.0), v, 0.0) for v in VTOP])
    ctx.set_source("Vd", vd)
    its = ctx.init_potential(tol=1e-12, max_iter=20000)
    return ctx, its


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


def cpu_baseline(nsteps=8):
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--refine-iters", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--only", choices=["refined", "fp64", "both"], default="both")
    a = ap.parse_args()
    if a.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(the step would shard by Fourier mode in 3D; see the design notes)", file=sys.stderr)
        sys.exit(2)
    import torch
    import paper_2305_09020_amd as pfd
    torch.cuda.set_device(0)
    res = {}
    for name, prec in (("refined", pfd.REFINED_FP32), ("fp64", pfd.PLAIN_FP64)):
        if a.only not in (name, "both"):
            continue
        ctx, its = make_context(prec, a.refine_iters)
        t = time_steps(ctx, a.steps, a.warmup)
        dof = ctx.planes * ctx.Nx * ctx.Ny
        res[name] = dict(t=t, dof=dof, value=dof * a.steps / t, ctx=ctx)
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
        "config": {"workload": "2D sessile drop, 20x20 elements order 8 (25,921 points), "
                               "rho 1:1000, mu 1:100, eps 1:40, V_top {0,0.5,1,2} as 4 instances, "
                               "dt 5e-5, closed box; %s path" % main_name,
                   "instances": len(VTOP), "dof_per_step": r["dof"],
                   "refine_iters": a.refine_iters if main_name == "refined" else 0},
    }
    if "fp64" in res and "refined" in res:
        out["fp64_value"] = res["fp64"]["value"]
        out["refined_over_fp64"] = res["refined"]["value"] / res["fp64"]["value"]
    if not a.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
