"""GPU parity: the HIP path (through the C-ABI) against the FP64 oracle, element by
element on the same seeded inputs.  Tolerances: plain FP64 path 1e-10 relative
per field (the oracle uses sparse LU, the library fast diagonalisation: both are
direct FP64 solves, differing by rounding); FP32-refined path 1e-8 (the
accuracy target of the refined path)."""
import math

import numpy as np
import pytest

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
from oracle.scheme import Scheme, Params, BCs, WALL, OPEN
from cases import mms_setup, mms_initial, mms_errors, c1_params
from gpu_cases import gpu_context, rel_err
from synth import drop_field

pytestmark = pytest.mark.gpu

FIELDS = ("phi", "psi", "V", "P", "ux", "uy", "Ex", "Ey")


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def box_case(n=4, K=6, periodic=False, top=WALL, par=None):
    xb = np.linspace(0.0, 1.0, n + 1)
    m = Mesh2D(xb, xb, K, periodic_x=periodic)
    side = {BOTTOM: WALL, TOP: top}
    if not periodic:
        side.update({LEFT: WALL, RIGHT: WALL})
    bc = BCs(side=side, pot_sides=(BOTTOM, TOP))
    return m, bc, par or c1_params()


# ------------------------------------------------------------------ solver (P8)
@pytest.mark.parametrize("periodic,top", [(False, WALL), (True, OPEN)])
@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_solve_matches_sparse_lu(periodic, top, precision, variant):
    """Each constant operator K + c M (families V, psi, phi, P, u) solved by the
    library matches SciPy's sparse LU of the assembled matrix on random data,
    with random Dirichlet values (remark after Algorithm 2)."""
    torch = _torch()
    m, bc, par = box_case(n=3, K=7, periodic=periodic, top=top)
    sch = Scheme(m, par, bc)
    ctx = gpu_context(m, par, bc, precision=precision)
    ctx.set_solver_variant(variant)
    rng = np.random.default_rng(230509020)
    tol = 1e-11 if precision == 0 else 1e-9
    for fam, name in enumerate(("V", "psi", "phi", "P", "u")):
        b = rng.standard_normal(m.Ng)
        g = rng.standard_normal(m.Ng)
        xr = sch.solve(name, 0, b, g)
        bt = torch.tensor(b, device="cuda")
        xt = torch.tensor(g, device="cuda")       # Dirichlet values + initial guess
        ctx.solve(fam, bt, xt)
        torch.cuda.synchronize()
        e = rel_err(xt.cpu().numpy(), xr)
        assert e < tol, (name, e)


@pytest.mark.parametrize("periodic,segs,top_dir", [
    (True, [(0.0, 1.0 / 3.0)], False),
    (True, [(0.0, 1.0 / 3.0), (2.0 / 3.0, 1.0)], True),
    (False, [(1.0 / 3.0, 2.0 / 3.0)], False),
])
@pytest.mark.parametrize("precision", [0, 1])
def test_potential_solve_with_electrode_segments(periodic, segs, top_dir, precision):
    """Potential operator with partial electrode segments on the bottom wall (Dirichlet on
    the segments, natural condition on the gaps, Sec. 5 test setups) against SciPy LU."""
    torch = _torch()
    n, K = 3, 7
    xb = np.linspace(0.0, 1.0, n + 1)
    m = Mesh2D(xb, xb, K, periodic_x=periodic)
    side = {BOTTOM: WALL, TOP: OPEN}
    if not periodic:
        side.update({LEFT: WALL, RIGHT: WALL})
    bc = BCs(side=side, pot_sides=(TOP,) if top_dir else (), electrodes=segs)
    par = c1_params()
    sch = Scheme(m, par, bc)
    assert 0 < len(sch.dir["V"]) < m.Nx + (m.Nx if top_dir else 0)
    ctx = gpu_context(m, par, bc, precision=precision)
    rng = np.random.default_rng(11)
    tol = 1e-11 if precision == 0 else 1e-9
    for trial in range(2):
        b = rng.standard_normal(m.Ng)
        g = rng.standard_normal(m.Ng)
        xr = sch.solve("V", 0, b, g)
        bt = torch.tensor(b, device="cuda")
        xt = torch.tensor(g, device="cuda")
        ctx.solve(0, bt, xt)
        torch.cuda.synchronize()
        e = rel_err(xt.cpu().numpy(), xr)
        assert e < tol, (trial, e)


# ------------------------------------------------------------- full-step parity
def run_pair(m, par, bc, phi0, u0, src, nsteps, nbatch=1, precision=0, equilibrium=False,
             per_step_src=None, init_V=True, V0=None, prev=None, P0=None, refine_max=0):
    """Run the oracle and the library side by side; returns list of (oracle, gpu) field dicts."""
    _torch()
    ctx = gpu_context(m, par, bc, nbatch=nbatch, precision=precision, refine_max=refine_max)
    schs = []
    for ib in range(nbatch):
        s = Scheme(m, par, bc)
        sl = (lambda a: None if a is None else np.asarray(a).reshape(nbatch, -1)[ib])
        s.set_state(sl(phi0), None if u0 is None else tuple(sl(x) for x in u0), sl(P0), sl(V0),
                    prev=None if prev is None else {k: (tuple(sl(x) for x in v) if k == "u" else sl(v))
                                                    for k, v in prev.items()})
        schs.append(s)
    shape = (nbatch, m.Ny, m.Nx)
    ctx.set_field("phi", np.reshape(phi0, shape))
    if u0 is not None:
        ctx.set_field("ux", np.reshape(u0[0], shape))
        ctx.set_field("uy", np.reshape(u0[1], shape))
    if P0 is not None:
        ctx.set_field("P", np.reshape(P0, shape))
    if V0 is not None:
        ctx.set_field("V", np.reshape(V0, shape))
    if prev is not None:
        for k in ("phi", "P", "V"):
            if k in prev:
                ctx.set_field(k, np.reshape(prev[k], shape), level=-1)
        if "u" in prev:
            ctx.set_field("ux", np.reshape(prev["u"][0], shape), level=-1)
            ctx.set_field("uy", np.reshape(prev["u"][1], shape), level=-1)
    ctx.set_sources({k: np.reshape(v, shape) for k, v in src.items()})
    if init_V:
        for ib, s in enumerate(schs):
            s.init_potential({k: np.reshape(v, (nbatch, -1))[ib] for k, v in src.items()})
        ctx.init_potential(tol=1e-14, max_iter=20000)
    out = []
    for n in range(nsteps):
        if per_step_src is not None:
            srcn = per_step_src(n)
            ctx.set_sources({k: np.reshape(v, shape) for k, v in srcn.items()})
        else:
            srcn = src
        o = [s.step({k: np.reshape(v, (nbatch, -1))[ib] for k, v in srcn.items()},
                    equilibrium=equilibrium) for ib, s in enumerate(schs)]
        ctx.step(1, equilibrium=equilibrium)
        gf = {k: ctx.get_field(k) for k in FIELDS}
        of = {k: np.stack([oo[k][0] for oo in o]).reshape(shape) for k in FIELDS}
        out.append((of, gf))
    return out, ctx


def check_parity(out, tol, fields=FIELDS, field_tol=None):
    """Per field, worst over the steps of the relative 2-norm error and of the element-wise
    error max|gpu - oracle| / max|oracle| (a wrong boundary row cannot hide in a norm);
    field_tol overrides tol."""
    worst = {}
    for (of, gf) in out:
        for k in fields:
            scale = max(np.linalg.norm(of[k]), 1e-12 * np.linalg.norm(of["phi"]))
            smax = max(np.abs(of[k]).max(), 1e-12 * np.abs(of["phi"]).max())
            e = max(np.linalg.norm(gf[k] - of[k]) / scale, np.abs(gf[k] - of[k]).max() / smax)
            worst[k] = max(worst.get(k, 0.0), e)
    lim = {k: (field_tol or {}).get(k, tol) for k in worst}
    print("parity", {k: "%.2e" % v for k, v in worst.items()})
    bad = {k: v for k, v in worst.items() if not v < lim[k]}
    assert not bad, (bad, worst)
    return worst


def test_c1_drop_step_parity_fp64():
    """C1 workload (4x4 elements, K = 6, drop r = 0.25, eta = 0.01, V 0/1): every
    field of Algorithm 1 after each of 10 steps."""
    m, bc, par = box_case(n=4, K=6)
    phi0 = drop_field(m.X, m.Y, (0.5, 0.5), 0.25, par.eta)
    vd = np.where(np.isclose(m.Y, 1.0), 1.0, 0.0)
    out, ctx = run_pair(m, par, bc, phi0, None, dict(Vd=vd), 10)
    check_parity(out, 1e-10)


@pytest.mark.parametrize("refine_max", [0, 8])
def test_c1_drop_step_parity_refined_fp32(refine_max):
    """Same with FP32 solves + FP64 iterative refinement to the backward-error stop rule
    (default and raised correction caps): 1e-8 per field."""
    m, bc, par = box_case(n=4, K=6)
    phi0 = drop_field(m.X, m.Y, (0.5, 0.5), 0.25, par.eta)
    vd = np.where(np.isclose(m.Y, 1.0), 1.0, 0.0)
    out, ctx = run_pair(m, par, bc, phi0, None, dict(Vd=vd), 10, precision=1, refine_max=refine_max)
    check_parity(out, 1e-8)


@pytest.mark.parametrize("precision,tol", [(0, 1e-9), (1, 1e-8)])
def test_benchmark_workload_parity(precision, tol):
    """The benchmark workload (20x20 elements, K = 8, sessile drop, rho 1:1000, mu 1:100,
    eps 1:40) at full size: two of its instances (V_top = 0.5 and 2) in one context,
    every field after each of 6 steps.  FP64 path 1e-9, FP32-refined path 1e-8.  The
    velocity starts from rest and is ~1e-5 after a
    few steps while the O(1-100) pressure and inertia terms of its equation nearly cancel,
    so rounding differences between the two FP64 implementations appear ~1e-9 relative
    to |u|: u is held to the 1e-8 bound on both paths."""
    from cases import c2_params
    from synth import C2
    par = c2_params()
    xb = np.linspace(0.0, 1.0, C2["nx"] + 1)
    m = Mesh2D(xb, xb, C2["K"])
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    phi1 = drop_field(m.X, m.Y, C2["center"], C2["r"], par.eta)
    vd = np.stack([np.where(np.isclose(m.Y, 1.0), v, 0.0) for v in (0.5, 2.0)])
    out, ctx = run_pair(m, par, bc, np.stack([phi1] * 2), None, dict(Vd=vd), 6, nbatch=2,
                        precision=precision)
    check_parity(out, tol, field_tol=dict(ux=1e-8, uy=1e-8))


def test_refinement_cap_reports_nonconvergence():
    """A correction cap the stop rule cannot be met within makes the step return PFD_ENOCONV
    (the state stays valid and the context usable); a tolerance that one FP32 correction
    meets does not.  The refinement record counts the failed solves."""
    import paper_2305_09020_amd as pfd
    _torch()
    m, bc, _ = box_case(n=4, K=6)
    par = c1_params()
    phi = drop_field(m.X, m.Y, (0.5, 0.3), 0.25, par.eta)
    vd = np.where(np.isclose(m.Y, 1.0), 1.0, 0.0)
    shape = (1, m.Ny, m.Nx)
    out = {}
    for label, rmax, rtol in (("cap1", 1, 0.0), ("loose", 1, 1e-6), ("default", 0, 0.0)):
        ctx = gpu_context(m, par, bc, precision=1, refine_max=rmax, refine_tol=rtol)
        ctx.set_field("phi", phi.reshape(shape))
        ctx.set_sources({"Vd": vd.reshape(shape)})
        ctx.init_potential(tol=1e-12, max_iter=2000)
        codes = []
        for n in range(4):
            try:
                ctx.step(1)
                codes.append(pfd.OK)
            except pfd.PfdError as e:
                codes.append(e.code)
        st = ctx.refine_stats()
        out[label] = (codes, st, {k: ctx.get_field(k) for k in ("phi", "ux")})
    codes, st, _ = out["cap1"]
    assert pfd.ENOCONV in codes, codes
    assert sum(s["failures"] for s in st) > 0
    codes, st, _ = out["loose"]
    assert codes == [pfd.OK] * 4, codes
    assert all(s["last_corrections"] <= 1 for s in st)
    codes, st, f = out["default"]
    assert codes == [pfd.OK] * 4, codes
    for fam, s in enumerate(st):
        if s["n_fp64_planes"] < 1:
            assert 1 <= s["last_corrections"] <= 4 and s["last_eta"] <= 1e-15, (fam, s)
    # the capped run's fields are still close to the converged ones
    assert rel_err(out["cap1"][2]["phi"], f["phi"]) < 1e-4


@pytest.mark.parametrize("nz", [0, 8])
def test_recycled_first_residual_matches_explicit(nz):
    """The refined path forms its first residual from the right sides of the two previous
    steps once they are recorded.  Against a twin context that is made to forget them before
    every step (re-setting a source, so every step computes the residual explicitly): the
    same fields to 1e-10 after 12 steps (2D closed box with walls and singular pressure; 3D
    periodic box with an open top), and the recycled context matches the FP64 path to 1e-8."""
    torch = _torch()
    if nz:
        xb = np.linspace(0.0, 1.0, 4)
        m = Mesh2D(xb, xb, 6, periodic_x=True)
        bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, pot_sides=(BOTTOM, TOP))
    else:
        m, bc, _ = box_case(n=4, K=6)
    par = c1_params()
    planes = nz if nz else 2
    X, Y = m.X.ravel()[None, :], m.Y.ravel()[None, :]
    Z = (np.arange(planes) / planes)[:, None] if nz else np.arange(planes)[:, None] * 0.05
    phi = np.tanh((np.sqrt((X - 0.5) ** 2 + (Y - 0.3) ** 2 + 0.1 * np.sin(2 * math.pi * Z) ** 2) - 0.25)
                  / (math.sqrt(2) * par.eta))
    vd = np.broadcast_to(np.where(np.isclose(Y, 1.0), 1.0, 0.0), phi.shape).copy()
    shape = (planes, m.Ny, m.Nx)
    ctxs = [gpu_context(m, par, bc, nbatch=1 if nz else planes, precision=p, nz=nz,
                        lz=1.0 if nz else 0.0) for p in (1, 1, 0)]
    ctxs[1].set_tuning(ctxs[0].tuning())
    for c in ctxs:
        c.set_field("phi", phi.reshape(shape))
        c.set_sources({"Vd": vd.reshape(shape)})
        c.init_potential(tol=1e-12, max_iter=2000)
    for n in range(12):
        ctxs[0].step(1)
        ctxs[1].set_sources({"Vd": vd.reshape(shape)})   # forgets the recorded right sides
        ctxs[1].step(1)
        ctxs[2].step(1)
    for k in ("phi", "psi", "V", "P", "ux", "uy"):
        a, b, f = (c.get_field(k) for c in ctxs)
        assert rel_err(a, b) < 1e-10, (k, rel_err(a, b))
        assert rel_err(a, f) < 1e-8, (k, rel_err(a, f))


def test_batched_instances_equal_oracle_runs():
    """Three instances in one context (one per plane) with different top
    voltages: each matches its own oracle run."""
    m, bc, par = box_case(n=3, K=5)
    phi1 = drop_field(m.X, m.Y, (0.5, 0.0), 0.3, 0.04)
    phi0 = np.stack([phi1] * 3)
    vd = np.stack([np.where(np.isclose(m.Y, 1.0), v, 0.0) for v in (0.0, 1.0, 2.0)])
    p2 = Params(**{**par.__dict__, "eta": 0.04, "lam": 3 * 0.04 / (2 * math.sqrt(2))})
    out, ctx = run_pair(m, p2, bc, phi0, None, dict(Vd=vd), 5, nbatch=3)
    check_parity(out, 1e-10)


def test_equilibrium_system_parity():
    """Simpler system of Sec. 2.4 (V, E, psi, phi with u = 0): parity and exact
    conservation of int_h phi on the GPU."""
    m, bc, par = box_case(n=3, K=6)
    p2 = Params(**{**par.__dict__, "eta": 0.04, "lam": 3 * 0.04 / (2 * math.sqrt(2)),
                   "theta_s_deg": 60.0, "dt": 1e-5})
    phi0 = drop_field(m.X, m.Y, (0.5, 0.0), 0.3, 0.04)
    vd = np.where(np.isclose(m.Y, 1.0), 2.0, 0.0)
    out, ctx = run_pair(m, p2, bc, phi0, None, dict(Vd=vd), 8, equilibrium=True)
    check_parity(out, 1e-10, fields=("phi", "psi", "V", "Ex", "Ey"))
    M = m.Mdiag
    m0 = np.sum(M * phi0.ravel())
    m1 = np.sum(M * out[-1][1]["phi"].ravel())
    assert abs(m1 - m0) < 1e-12 * abs(m0)


@pytest.mark.parametrize("kind", ["eq80", "box"])
def test_manufactured_parity_and_accuracy(kind):
    """Manufactured solutions (Sec. 4.1 eq. 80; closed box): the GPU path matches
    the oracle step by step with time-dependent sources, and its error against
    the exact solution is the oracle's."""
    K, dt, n = 8, 1e-3, 20
    case = mms_setup(kind, K, dt)
    m, par, bc = case["mesh"], case["par"], case["bc"]
    f0, fm = mms_initial(case, dt)
    x, y, z = case["x"], case["y"], case["z"]
    mf = case["mf"]
    src_fn = lambda i: mf.sources(x, y, z, (i + 1) * dt, case["sides"])
    out, ctx = run_pair(m, par, bc, f0["phi"], f0["u"][:2], src_fn(0), n, per_step_src=src_fn,
                        init_V=False, V0=f0["V"], P0=f0["P"],
                        prev=dict(phi=fm["phi"], u=fm["u"][:2], P=fm["P"], V=fm["V"]))
    check_parity(out, 1e-10)
    of, gf = out[-1]
    fe = mf.fields(x, y, z, n * dt)
    eg = max(np.max(np.abs(gf["phi"].ravel() - fe["phi"].ravel())),
             np.max(np.abs(gf["ux"].ravel() - fe["u"][0].ravel())))
    assert eg < 1e-3


def test_init_potential_matches_direct_solve():
    """Remark 3.1 fixed point on the GPU converges to the oracle's direct
    variable-coefficient solve."""
    m, bc, par = box_case(n=4, K=6)
    phi0 = drop_field(m.X, m.Y, (0.5, 0.5), 0.25, par.eta)
    vd = np.where(np.isclose(m.Y, 1.0), 1.0, 0.0)
    sch = Scheme(m, par, bc)
    sch.set_state(phi0.ravel())
    Vo = sch.init_potential(dict(Vd=vd.ravel()))
    ctx = gpu_context(m, par, bc)
    ctx.set_field("phi", phi0.reshape(1, m.Ny, m.Nx))
    ctx.set_source("Vd", vd.reshape(1, m.Ny, m.Nx))
    its = ctx.init_potential(tol=1e-14, max_iter=5000)
    assert its < 5000
    Vg = ctx.get_field("V")
    assert rel_err(Vg, Vo) < 1e-12


def test_nonfinite_state_is_reported():
    """A NaN written into the state is caught by the step's guard (sticky error)."""
    import paper_2305_09020_amd as pfd
    m, bc, par = box_case(n=2, K=4)
    ctx = gpu_context(m, par, bc)
    phi = drop_field(m.X, m.Y, (0.5, 0.5), 0.25, 0.05).reshape(1, m.Ny, m.Nx).copy()
    phi[0, 3, 3] = np.nan
    ctx.set_field("phi", phi)
    with pytest.raises(pfd.PfdError) as ei:
        ctx.step(1)
    assert ei.value.code == pfd.ENONFINITE
    with pytest.raises(pfd.PfdError) as ei:
        ctx.step(1)
    assert ei.value.code == pfd.ESTATE


@pytest.mark.parametrize("precision", [0, 1])
def test_solver_variants_agree_on_benchmark_shapes(precision):
    """The fast-diagonalisation kernel variants (four GEMM passes; fused strips; fused middle
    passes) on the benchmark configuration's shapes (4 planes of 161 x 161, K = 8): the same
    solution of every family up to rounding, and the autotuner's choice is one of them."""
    torch = _torch()
    from synth import C2, c2_param_dict
    import paper_2305_09020_amd as pfd
    xb = np.linspace(0.0, 1.0, C2["nx"] + 1)
    prob = pfd.make_problem(xb, xb, C2["K"], c2_param_dict(), [pfd.WALL] * 4, [1, 1, 0, 0], nbatch=4,
                            precision=precision)
    ctx = pfd.Context(prob)
    v, us = ctx.solver_variant()
    assert v in (0, 1, 2) and us[0] > 0 and us[1] > 0 and us[2] > 0
    rng = np.random.default_rng(3)
    n = ctx.planes * ctx.Ny * ctx.Nx
    for fam in range(5):
        b = torch.tensor(rng.standard_normal(n), device="cuda")
        g = torch.tensor(rng.standard_normal(n), device="cuda")
        out = []
        for var in (0, 1, 2):
            ctx.set_solver_variant(var)
            x = g.clone()
            ctx.solve(fam, b, x)
            out.append(x.cpu().numpy())
        for var in (1, 2):
            e = rel_err(out[var], out[0])
            assert e < (1e-12 if precision == 0 else 1e-9), (fam, var, e)


@pytest.mark.parametrize("tg,p1", [(0, 0), (1, 0), (2, 0), (3, 0), (4, 0), (5, 0), (6, 0), (0, 1), (5, 1)])
def test_refined_last_pass_every_width(tg, p1):
    """Refined solves with the fused middle passes and each form of the last pass (GEMM; the
    padded-row matrix-core kernel with 1-4 column tiles per wave, and with one tile and
    four-slice fragment chunks; the kernel with Sx resident in LDS) and of the first pass
    (GEMM; Sx resident in LDS) match SciPy's sparse LU for every
    family on a 3-plane batch (Nx = 41: three column tiles, the last one ragged)."""
    torch = _torch()
    m, bc, par = box_case(n=5, K=8, periodic=True, top=OPEN)
    sch = Scheme(m, par, bc)
    ctx = gpu_context(m, par, bc, nbatch=3, precision=1)
    t = ctx.tuning()
    assert len(t) == 15
    t[10] = 2      # fused middle passes
    t[13] = tg     # last pass
    t[14] = p1     # first pass
    ctx.set_tuning(t)
    assert ctx.tuning() == t
    rng = np.random.default_rng(37 + tg)
    for fam, name in enumerate(("V", "psi", "phi", "P", "u")):
        b = rng.standard_normal((3, m.Ng))
        g = rng.standard_normal((3, m.Ng))
        xr = np.stack([sch.solve(name, 0, b[i], g[i]) for i in range(3)])
        xt = torch.tensor(g.ravel(), device="cuda")
        ctx.solve(fam, torch.tensor(b.ravel(), device="cuda"), xt)
        torch.cuda.synchronize()
        assert rel_err(xt.cpu().numpy(), xr) < 1e-9, (name, rel_err(xt.cpu().numpy(), xr))


@pytest.mark.parametrize("precision", [0, 1])
def test_fused_middle_passes_tall_mesh(precision):
    """A mesh with Ny = 265 (more than 16 row tiles, so a wave of the fused middle-pass
    kernel takes two; in FP64 its LDS block does not fit and the variant falls back to the
    four passes): every family solves to the sparse-LU solution with variant 2."""
    torch = _torch()
    xb = np.linspace(0.0, 0.2, 3)
    yb = np.linspace(0.0, 1.0, 34)
    m = Mesh2D(xb, yb, 8, periodic_x=False)
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    par = c1_params()
    sch = Scheme(m, par, bc)
    ctx = gpu_context(m, par, bc, precision=precision)
    assert ctx.Ny == 265
    ctx.set_solver_variant(2)
    rng = np.random.default_rng(29)
    tol = 1e-11 if precision == 0 else 1e-9
    for fam, name in enumerate(("V", "psi", "phi", "P", "u")):
        b = rng.standard_normal(m.Ng)
        g = rng.standard_normal(m.Ng)
        xr = sch.solve(name, 0, b, g)
        bt = torch.tensor(b, device="cuda")
        xt = torch.tensor(g, device="cuda")
        ctx.solve(fam, bt, xt)
        torch.cuda.synchronize()
        assert rel_err(xt.cpu().numpy(), xr) < tol, (name, rel_err(xt.cpu().numpy(), xr))


@pytest.mark.parametrize("precision", [0, 1])
def test_every_gemm_tile_configuration_solves(precision):
    """Each tile configuration of the batched GEMM (forced at all call sites, four-pass
    solver) solves every family to the sparse-LU solution; the autotuner's timings cover
    every configuration of the four passes."""
    torch = _torch()
    m, bc, par = box_case(n=3, K=7, periodic=True, top=OPEN)
    sch = Scheme(m, par, bc)
    ctx = gpu_context(m, par, bc, precision=precision)
    cfg, us = ctx.gemm_config()
    assert all(0 <= c < 16 for c in cfg)
    assert all(t > 0 for site in range(4) for t in us[site][:8])
    assert all(len(u) == 17 for u in us)
    ctx.set_solver_variant(0)
    rng = np.random.default_rng(17)
    tol = 1e-11 if precision == 0 else 1e-9
    cases = []
    for fam, name in enumerate(("V", "psi", "phi", "P", "u")):
        b = rng.standard_normal(m.Ng)
        g = rng.standard_normal(m.Ng)
        cases.append((fam, b, g, sch.solve(name, 0, b, g)))
    for c in range(16):
        ctx.set_gemm_config(-1, c)
        for fam, b, g, xr in cases:
            xt = torch.tensor(g, device="cuda")
            ctx.solve(fam, torch.tensor(b, device="cuda"), xt)
            torch.cuda.synchronize()
            e = rel_err(xt.cpu().numpy(), xr)
            assert e < tol, (c, fam, e)


@pytest.mark.parametrize("periodic", [False, True])
def test_residual_kernel_variants_identical(periodic):
    """The residual kernels (per-node; LDS-tiled rows; per-node with the order a runtime
    argument) give the same refined solves (same sums in the same order; only the compiler's
    fused multiply-adds may differ) and the autotuner timed the first two."""
    torch = _torch()
    m, bc, par = box_case(n=5, K=8, periodic=periodic, top=OPEN if periodic else WALL)
    ctx = gpu_context(m, par, bc, nbatch=3, precision=1)
    v, us = ctx.residual_variant()
    assert v in (0, 1, 2) and us[0] > 0 and us[1] > 0
    rng = np.random.default_rng(9)
    n = ctx.planes * m.Ng
    for fam in range(5):
        b = torch.tensor(rng.standard_normal(n), device="cuda")
        g = torch.tensor(rng.standard_normal(n), device="cuda")
        out = []
        for var in (0, 1, 3):
            ctx.set_residual_variant(var)
            x = g.clone()
            ctx.solve(fam, b, x)
            out.append(x.cpu().numpy())
        assert rel_err(out[1], out[0]) < 1e-13, (fam, rel_err(out[1], out[0]))
        assert rel_err(out[2], out[0]) < 1e-13, (fam, rel_err(out[2], out[0]))


@pytest.mark.parametrize("periodic,top", [(False, WALL), (True, OPEN)])
@pytest.mark.parametrize("solver", [0, 2])
def test_fused_residual_first_pass_solves(periodic, top, solver):
    """Refined solves with the residual fused with the first fast-diagonalisation pass
    (residual variant 2, with the four-pass and the fused-middle solvers) match SciPy's
    sparse LU for every family on a 3-plane batch, and agree with the separate residual to
    the refinement's rounding; the singular pressure (walls) takes the separate residual."""
    torch = _torch()
    m, bc, par = box_case(n=5, K=8, periodic=periodic, top=top)
    sch = Scheme(m, par, bc)
    ctx = gpu_context(m, par, bc, nbatch=3, precision=1)
    ctx.set_solver_variant(solver)
    rng = np.random.default_rng(31)
    for fam, name in enumerate(("V", "psi", "phi", "P", "u")):
        b = rng.standard_normal((3, m.Ng))
        g = rng.standard_normal((3, m.Ng))
        xr = np.stack([sch.solve(name, 0, b[i], g[i]) for i in range(3)])
        out = []
        for var in (1, 2):
            ctx.set_residual_variant(var)
            xt = torch.tensor(g.ravel(), device="cuda")
            ctx.solve(fam, torch.tensor(b.ravel(), device="cuda"), xt)
            torch.cuda.synchronize()
            out.append(xt.cpu().numpy())
        assert rel_err(out[1], xr) < 1e-9, (name, rel_err(out[1], xr))
        assert rel_err(out[1], out[0]) < 1e-9, (name, rel_err(out[1], out[0]))
