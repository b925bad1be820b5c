"""GPU parity of the 3D path (Algorithm 2: spectral elements in x-y, Fourier in z)
against the oracle's per-mode solves, on the same seeded inputs."""
import math

import numpy as np
import pytest

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT
from oracle.scheme import Scheme, Params, BCs, WALL, OPEN
from cases import mms_setup, mms_initial, c1_params
from gpu_cases import gpu_context, rel_err
from synth import drop_field

pytestmark = pytest.mark.gpu

FIELDS3 = ("phi", "psi", "V", "P", "ux", "uy", "uz", "Ex", "Ey", "Ez")


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def box3d(n=2, K=5, Nz=8, Lz=1.0, top=WALL, periodic=False):
    xb = np.linspace(0.0, 1.0, n + 1)
    m = Mesh2D(xb, xb, K, periodic_x=periodic)
    side = {BOTTOM: WALL, TOP: top}
    if not periodic:
        side.update({LEFT: WALL, RIGHT: WALL})
    bc = BCs(side=side, pot_sides=(BOTTOM, TOP))
    return m, bc


def packed_mode(p, Nz):
    """(mode k, part) of packed spectral plane p: part 0 = real, 1 = imaginary."""
    if p == 0:
        return 0, 0
    if p == 1:
        return Nz // 2, 0
    return p // 2, p % 2


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_3d_mode_solves_match_sparse_lu(precision, variant):
    """Every per-mode operator K + (c_f + beta_k^2) M (eqs. 74-78), including the k = 0
    singular pressure and the Nyquist mode, against SciPy LU on random data."""
    torch = _torch()
    Nz, Lz = 8, 1.7
    m, bc = box3d(n=3, K=6, Nz=Nz, Lz=Lz, top=OPEN, periodic=True)
    par = c1_params()
    sch = Scheme(m, par, bc, Nz=Nz, Lz=Lz)
    ctx = gpu_context(m, par, bc, nz=Nz, lz=Lz, precision=precision)
    ctx.set_solver_variant(variant)
    rng = np.random.default_rng(7)
    tol = 1e-11 if precision == 0 else 1e-9
    for fam, name in enumerate(("V", "psi", "phi", "P", "u")):
        b = rng.standard_normal((Nz, m.Ng))
        gd = rng.standard_normal((Nz, m.Ng))
        ref = np.zeros((Nz, m.Ng))
        for p in range(Nz):
            k, part = packed_mode(p, Nz)
            ref[p] = sch.solve(name, k, b[p], gd[p])
        bt = torch.tensor(b, device="cuda")
        xt = torch.tensor(gd, device="cuda")
        ctx.solve(fam, bt, xt)
        torch.cuda.synchronize()
        e = rel_err(xt.cpu().numpy(), ref)
        assert e < tol, (name, e)


@pytest.mark.parametrize("precision", [0, 1])
def test_3d_potential_mode_solves_with_electrodes(precision):
    """Per-mode potential operators K + beta_k^2 M with a partial electrode segment on the
    bottom wall (gap nodes unknown in every mode) against SciPy LU."""
    torch = _torch()
    Nz, Lz = 8, 1.7
    xb = np.linspace(0.0, 1.0, 4)
    m = Mesh2D(xb, xb, 6, periodic_x=True)
    bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, electrodes=[(1.0 / 3.0, 2.0 / 3.0)])
    par = c1_params()
    sch = Scheme(m, par, bc, Nz=Nz, Lz=Lz)
    ctx = gpu_context(m, par, bc, nz=Nz, lz=Lz, precision=precision)
    rng = np.random.default_rng(8)
    tol = 1e-11 if precision == 0 else 1e-9
    b = rng.standard_normal((Nz, m.Ng))
    gd = rng.standard_normal((Nz, m.Ng))
    ref = np.zeros((Nz, m.Ng))
    for p in range(Nz):
        k, part = packed_mode(p, Nz)
        ref[p] = sch.solve("V", k, b[p], gd[p])
    bt = torch.tensor(b, device="cuda")
    xt = torch.tensor(gd, device="cuda")
    ctx.solve(0, bt, xt)
    torch.cuda.synchronize()
    e = rel_err(xt.cpu().numpy(), ref)
    assert e < tol, e


def run3d(m, bc, par, Nz, Lz, phi0, u0, src, nsteps, precision=0, equilibrium=False,
          per_step_src=None, V0=None, P0=None, prev=None, init_V=True):
    _torch()
    ctx = gpu_context(m, par, bc, nz=Nz, lz=Lz, precision=precision)
    sch = Scheme(m, par, bc, Nz=Nz, Lz=Lz)
    sch.set_state(phi0, u0, P0, V0, prev=prev)
    shape = (Nz, m.Ny, m.Nx)
    ctx.set_field("phi", np.reshape(phi0, shape))
    if u0 is not None:
        for k, v in zip(("ux", "uy", "uz"), u0):
            ctx.set_field(k, np.reshape(v, shape))
    if P0 is not None:
        ctx.set_field("P", np.reshape(P0, shape))
    if V0 is not None:
        ctx.set_field("V", np.reshape(V0, shape))
    if prev is not None:
        for k in ("phi", "P", "V"):
            ctx.set_field(k, np.reshape(prev[k], shape), level=-1)
        for k, v in zip(("ux", "uy", "uz"), prev["u"]):
            ctx.set_field(k, np.reshape(v, shape), level=-1)
    ctx.set_sources({k: np.reshape(v, shape) for k, v in src.items()})
    if init_V:
        sch.init_potential(src)
        ctx.init_potential(tol=1e-13, max_iter=20000)
    out = []
    for n in range(nsteps):
        srcn = src if per_step_src is None else per_step_src(n)
        if per_step_src is not None:
            ctx.set_sources({k: np.reshape(v, shape) for k, v in srcn.items()})
        o = sch.step(srcn, equilibrium=equilibrium)
        ctx.step(1, equilibrium=equilibrium)
        out.append(({k: o[k] for k in FIELDS3}, {k: ctx.get_field(k).reshape(Nz, -1) for k in FIELDS3}))
    return out, ctx


def check(out, tol, fields=FIELDS3, field_tol=None):
    """Per field, worst over the steps of the relative 2-norm error and of the element-wise
    error max|gpu - oracle| / max|oracle| (a wrong boundary row cannot hide in a norm)."""
    worst = {}
    for of, gf in out:
        for k in fields:
            scale = max(np.linalg.norm(of[k]), 1e-12 * np.linalg.norm(of["phi"]))
            smax = max(np.abs(of[k]).max(), 1e-12 * np.abs(of["phi"]).max())
            e = max(np.linalg.norm(gf[k] - of[k]) / scale, np.abs(gf[k] - of[k]).max() / smax)
            worst[k] = max(worst.get(k, 0.0), e)
    print("parity", {k: "%.2e" % v for k, v in worst.items()})
    lim = {k: (field_tol or {}).get(k, tol) for k in worst}
    bad = {k: v for k, v in worst.items() if not v < lim[k]}
    assert not bad, (bad, worst)


def _ellipsoid(m, Nz, Lz, eta):
    z = np.arange(Nz) * Lz / Nz
    X = np.broadcast_to(m.X.ravel()[None, :], (Nz, m.Ng))
    Y = np.broadcast_to(m.Y.ravel()[None, :], (Nz, m.Ng))
    Z = np.broadcast_to(z[:, None], (Nz, m.Ng))
    d = np.sqrt((X - 0.5) ** 2 + (Y - 0.3) ** 2 + 0.5 * (Z - 0.5) ** 2)
    return np.tanh((d - 0.3) / (math.sqrt(2) * eta))


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-8)])
def test_3d_drop_step_parity(precision, tol):
    """A z-varying drop in a closed box (walls, V = 0 / 1 bottom / top, Nz = 8): every field of
    Algorithm 2 after each of 4 steps."""
    Nz, Lz = 8, 1.0
    m, bc = box3d(n=2, K=5, Nz=Nz, Lz=Lz)
    par = Params(**{**c1_params().__dict__, "eta": 0.05, "lam": 3 * 0.05 / (2 * math.sqrt(2)),
                    "theta_s_deg": 70.0})
    phi0 = _ellipsoid(m, Nz, Lz, par.eta)
    vd = np.broadcast_to(np.where(np.isclose(m.Y.ravel(), 1.0), 1.0, 0.0)[None, :], (Nz, m.Ng)).copy()
    rng = np.random.default_rng(3)
    u0 = tuple(0.05 * np.sin(np.pi * m.X.ravel())[None, :] * np.sin(np.pi * m.Y.ravel())[None, :]
               * np.cos(2 * np.pi * (np.arange(Nz)[:, None] / Nz + 0.1 * i)) for i in range(3))
    out, ctx = run3d(m, bc, par, Nz, Lz, phi0, u0, dict(Vd=vd), 4, precision=precision)
    check(out, tol)


def test_3d_equilibrium_parity_and_mass():
    """Equilibrium system in 3D: parity and conservation of int_h phi (k = 0 mode)."""
    Nz, Lz = 8, 1.0
    m, bc = box3d(n=2, K=5, Nz=Nz, Lz=Lz)
    par = Params(**{**c1_params().__dict__, "eta": 0.05, "lam": 3 * 0.05 / (2 * math.sqrt(2)),
                    "theta_s_deg": 60.0, "dt": 1e-5})
    phi0 = _ellipsoid(m, Nz, Lz, par.eta)
    vd = np.broadcast_to(np.where(np.isclose(m.Y.ravel(), 1.0), 2.0, 0.0)[None, :], (Nz, m.Ng)).copy()
    out, ctx = run3d(m, bc, par, Nz, Lz, phi0, None, dict(Vd=vd), 4, equilibrium=True)
    check(out, 1e-10, fields=("phi", "psi", "V", "Ex", "Ey", "Ez"))
    m0 = np.sum(phi0 * m.Mdiag[None, :])
    m1 = np.sum(out[-1][1]["phi"] * m.Mdiag[None, :])
    assert abs(m1 - m0) < 1e-12 * abs(m0)


def test_3d_manufactured_parity():
    """eq. (81) manufactured solution (V Dirichlet on the whole bottom wall), Nz = 8, K = 6,
    open top: parity with the oracle step by step with time-dependent sources."""
    K, dt, n = 6, 1e-3, 6
    case = mms_setup("eq81b", K, dt, Nz=8)
    m, par, bc = case["mesh"], case["par"], case["bc"]
    f0, fm = mms_initial(case, dt)
    x, y, z = case["x"], case["y"], case["z"]
    mf = case["mf"]
    src_fn = lambda i: mf.sources(x, y, z, (i + 1) * dt, case["sides"])
    out, ctx = run3d(m, bc, par, 8, 2.0, f0["phi"], f0["u"], src_fn(0), n, per_step_src=src_fn,
                     V0=f0["V"], P0=f0["P"], init_V=False,
                     prev=dict(phi=fm["phi"], u=fm["u"], P=fm["P"], V=fm["V"]))
    check(out, 1e-10)


def test_3d_manufactured_parity_electrode():
    """eq. (81) manufactured solution with its electrode on x in [0, 1] of the bottom wall
    and the natural condition on x in (1, 2): parity with the oracle step by step."""
    K, dt, n = 6, 1e-3, 6
    case = mms_setup("eq81", K, dt, Nz=8)
    m, par, bc = case["mesh"], case["par"], case["bc"]
    assert bc.electrodes
    f0, fm = mms_initial(case, dt)
    x, y, z = case["x"], case["y"], case["z"]
    mf = case["mf"]
    src_fn = lambda i: mf.sources(x, y, z, (i + 1) * dt, case["sides"])
    out, ctx = run3d(m, bc, par, 8, 2.0, f0["phi"], f0["u"], src_fn(0), n, per_step_src=src_fn,
                     V0=f0["V"], P0=f0["P"], init_V=False,
                     prev=dict(phi=fm["phi"], u=fm["u"], P=fm["P"], V=fm["V"]))
    check(out, 1e-10)


@pytest.mark.parametrize("cfg", list(range(17)))
def test_3d_z_transform_every_tile_configuration(cfg):
    """The z transforms with each GEMM configuration of the packed DFT matrices forced
    (0..15), and with the batched FFT (16): 3D equilibrium steps still match the
    oracle (forward, inverse and both derivative transforms are used)."""
    _torch()
    Nz, Lz = 8, 1.0
    m, bc = box3d(n=2, K=5, Nz=Nz, Lz=Lz)
    par = c1_params()
    phi0 = _ellipsoid(m, Nz, Lz, par.eta)
    vd = np.broadcast_to(np.where(np.isclose(m.Y.ravel(), 1.0), 2.0, 0.0)[None, :], (Nz, m.Ng)).copy()
    ctx0 = gpu_context(m, par, bc, nz=Nz, lz=Lz)
    ctx0.set_gemm_config(4, cfg)
    sch = Scheme(m, par, bc, Nz=Nz, Lz=Lz)
    sch.set_state(phi0)
    shape = (Nz, m.Ny, m.Nx)
    ctx0.set_field("phi", phi0.reshape(shape))
    ctx0.set_sources({"Vd": vd.reshape(shape)})
    sch.init_potential(dict(Vd=vd))
    ctx0.init_potential(tol=1e-13, max_iter=20000)
    for n in range(2):
        o = sch.step(dict(Vd=vd), equilibrium=True)
        ctx0.step(1, equilibrium=True)
    for k in ("phi", "V", "Ez"):
        ref = o[k]
        got = ctx0.get_field(k).reshape(Nz, -1)
        assert rel_err(got, ref) < 1e-10, (k, rel_err(got, ref))


@pytest.mark.parametrize("nz,n", [(4, 2), (16, 2), (64, 2), (128, 4), (256, 3)])
def test_3d_fft_equals_dft_gemm(nz, n):
    """Full steps with the FFT and with the dense-DFT GEMM on the same context agree to
    rounding (power-of-two plane counts; closed box, drop; 81, 289 and 169 nodes per plane,
    so the last FFT work-group is partly empty)."""
    torch = _torch()
    Lz = 1.3
    m, bc = box3d(n=n, K=4, Nz=nz, Lz=Lz)
    par = c1_params()
    phi0 = _ellipsoid(m, nz, Lz, par.eta)
    vd = np.broadcast_to(np.where(np.isclose(m.Y.ravel(), 1.0), 1.0, 0.0)[None, :], (nz, m.Ng)).copy()
    shape = (nz, m.Ny, m.Nx)
    res = []
    for cfg in (0, 16):
        ctx = gpu_context(m, par, bc, nz=nz, lz=Lz)
        ctx.set_gemm_config(4, cfg)
        ctx.set_field("phi", phi0.reshape(shape))
        ctx.set_sources({"Vd": vd.reshape(shape)})
        ctx.init_potential(tol=1e-13, max_iter=20000)
        ctx.step(3)
        res.append({k: ctx.get_field(k) for k in ("phi", "V", "P", "ux", "uz", "Ez")})
    for k in res[0]:
        assert rel_err(res[1][k], res[0][k]) < 1e-11, (k, rel_err(res[1][k], res[0][k]))


_ORACLE_CACHE = {}


def _case_128():
    """The 128-plane, order-8 case and the oracle's fields after each of 3 steps (computed once
    per test session: they do not depend on the GPU settings under test)."""
    if "c128" in _ORACLE_CACHE:
        return _ORACLE_CACHE["c128"]
    Nz, Lz = 128, 2.0
    m, bc = box3d(n=2, K=8, Nz=Nz, Lz=Lz)
    par = Params(**{**c1_params().__dict__, "eta": 0.05, "lam": 3 * 0.05 / (2 * math.sqrt(2)),
                    "theta_s_deg": 80.0, "rho2": 10.0})
    z = np.arange(Nz) * Lz / Nz
    X = np.broadcast_to(m.X.ravel()[None, :], (Nz, m.Ng))
    Y = np.broadcast_to(m.Y.ravel()[None, :], (Nz, m.Ng))
    Z = np.broadcast_to(z[:, None], (Nz, m.Ng))
    r = 0.3 * (1.0 + 0.05 * np.cos(2 * np.pi * X) * np.cos(2 * np.pi * Z / Lz + 0.3))
    phi0 = np.tanh((np.sqrt((X - 0.5) ** 2 + (Y - 0.5) ** 2 + (Z - 1.0) ** 2) - r) / (math.sqrt(2) * par.eta))
    u0 = tuple(0.02 * np.sin(np.pi * X) * np.sin(np.pi * Y) * np.cos(2 * np.pi * (Z / Lz + 0.2 * i))
               for i in range(3))
    vd = np.where(np.isclose(Y, 1.0), 1.0, 0.0)
    sch = Scheme(m, par, bc, Nz=Nz, Lz=Lz)
    sch.set_state(phi0, u0)
    sch.init_potential(dict(Vd=vd))
    ref = []
    for n in range(3):
        o = sch.step(dict(Vd=vd))
        ref.append({k: np.array(o[k]) for k in FIELDS3})
    _ORACLE_CACHE["c128"] = (m, bc, par, Nz, Lz, phi0, u0, vd, ref)
    return _ORACLE_CACHE["c128"]


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-8)])
@pytest.mark.parametrize("variant", [0, 1, 2])
def test_3d_128_planes_order_8_parity(precision, tol, variant):
    """The plane count and order of the 3D benchmark workload (Nz = 128, K = 8, so the
    128-point z FFT and the order-8 residual and fast-diagonalisation kernels run) on a
    small 2x2-element box: a perturbed sphere with an initial velocity, walls, V 0 / 1; every
    field of Algorithm 2 against the oracle after each of 3 steps, per element, with each
    fast-diagonalisation variant and the batched FFT in z."""
    _torch()
    m, bc, par, Nz, Lz, phi0, u0, vd, ref = _case_128()
    ctx = gpu_context(m, par, bc, nz=Nz, lz=Lz, precision=precision)
    ctx.set_solver_variant(variant)
    ctx.set_gemm_config(4, 16)
    shape = (Nz, m.Ny, m.Nx)
    ctx.set_field("phi", phi0.reshape(shape))
    for k, v in zip(("ux", "uy", "uz"), u0):
        ctx.set_field(k, np.ascontiguousarray(v).reshape(shape))
    ctx.set_sources({"Vd": vd.reshape(shape)})
    ctx.init_potential(tol=1e-13, max_iter=20000)
    out = []
    for n in range(3):
        ctx.step(1)
        out.append((ref[n], {k: ctx.get_field(k).reshape(Nz, -1) for k in FIELDS3}))
    check(out, tol)


@pytest.mark.parametrize("precision,tol", [(0, 1e-10), (1, 1e-8)])
def test_3d_64_planes_electrode_equilibrium_parity(precision, tol):
    """The plane count, order and boundary family of the learned-warm-start workload (Nz = 64,
    K = 6, x-periodic, open top, bottom electrodes cycling +V, gap, -V, gap over the
    x-elements, contact angle 70 deg) on a 4x2-element box: the equilibrium system (eq. 16)
    against the oracle after each of 4 steps, per element (64-point FFT, electrode gap solves
    in every mode)."""
    _torch()
    Nz, Lz = 64, 1.0
    xb = np.linspace(0.0, 1.0, 5)
    yb = np.linspace(0.0, 0.5, 3)
    m = Mesh2D(xb, yb, 6, periodic_x=True)
    el = [(0.0, 0.25), (0.5, 0.75)]
    bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, electrodes=el)
    par = Params(**{**c1_params().__dict__, "eta": 0.04, "lam": 3 * 0.04 / (2 * math.sqrt(2)),
                    "theta_s_deg": 70.0, "eps1": 1e-3, "eps2": 4e-3, "dt": 5e-5})
    z = np.arange(Nz) * Lz / Nz
    X = np.broadcast_to(m.X.ravel()[None, :], (Nz, m.Ng))
    Y = np.broadcast_to(m.Y.ravel()[None, :], (Nz, m.Ng))
    Z = np.broadcast_to(z[:, None], (Nz, m.Ng))
    phi0 = np.tanh((np.sqrt((X - 0.5) ** 2 + Y ** 2 + (Z - 0.5) ** 2) - 0.25) / (math.sqrt(2) * par.eta))
    bottom = np.isclose(Y, 0.0)
    vd = np.where(bottom & (X <= 0.25 + 1e-12), 1.5, 0.0) + np.where(bottom & (X >= 0.5 - 1e-12) & (X <= 0.75 + 1e-12), -1.5, 0.0)
    out, ctx = run3d(m, bc, par, Nz, Lz, phi0, None, dict(Vd=vd), 4, precision=precision, equilibrium=True)
    check(out, tol, fields=("phi", "psi", "V", "Ex", "Ey", "Ez"))
