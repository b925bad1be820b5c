"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  This module holds workload descriptions (mesh sizes, material
parameters, boundary sides) and initial-condition generators only -- none of the
method's arithmetic.  Fields are evaluated on coordinates supplied by the caller.

Workloads follow the paper's setups (tanh interface profiles of a drop in an
ambient fluid, Sec. 4.2-4.4) at the sizes of the benchmark configurations:
  C1  [0,1]^2, 4x4 elements, K = 6, dt = 1e-4, 100 steps, drop r = 0.25 at the
      centre, eta = 0.01, rho 1:2, mu 0.01:0.02, eps 2:8, walls, V = 0 / 1 on the
      bottom / top.
  C2  [0,1]^2, 20x20 elements, K = 8, dt = 5e-5, 2000 steps, sessile half-disc
      r = 0.25 at (0.5, 0), theta_s = 90 deg, eta = 0.01, rho 1:1000,
      mu 0.01:1, eps 1:40, V_top in {0, 0.5, 1, 2} (four instances).
  C3  [0,1]^2 x [0, 2) (z periodic), 16x16 elements, K = 8, Nz = 128, dt = 1e-4, 500
      steps, sphere r = 0.3 at (0.5, 0.5, 1.0) with a 1% radius perturbation
      r = 0.3 (1 + 0.01 xi(x)), xi = sum of 8 cosines with integer wave vectors and
      amplitudes / phases drawn from numpy PCG64 (seed 230509020), amplitudes
      normalised to sum 1 (so |xi| <= 1); eta = 0.02, rho 1:10, mu 0.01:0.02,
      eps 0.1:1 (ratio 10), walls, V = 0 / 1 on the bottom / top.
Fluid 1 (phi = +1) is the ambient fluid, fluid 2 (phi = -1) the drop.
"""
import math

import numpy as np


def lam_from_sigma(sigma, eta):
    """lambda = 3 sigma eta / (2 sqrt 2), the relation quoted in Sec. 2.1."""
    return 3.0 * sigma * eta / (2.0 * math.sqrt(2.0))


def drop_field(X, Y, center, r, eta, Z=None, zc=None, rfun=None):
    """phi = tanh((|x - c| - r)/(sqrt(2) eta)): -1 inside the drop, +1 outside."""
    d2 = (np.asarray(X) - center[0]) ** 2 + (np.asarray(Y) - center[1]) ** 2
    if Z is not None:
        d2 = d2 + (np.asarray(Z) - zc) ** 2
    rr = r if rfun is None else rfun
    return np.tanh((np.sqrt(d2) - rr) / (math.sqrt(2.0) * eta))


def c1_param_dict(dt=1e-4):
    eta = 0.01
    return dict(rho1=1.0, rho2=2.0, mu1=0.01, mu2=0.02, eps1=2.0, eps2=8.0,
                lam=lam_from_sigma(1.0, eta), eta=eta, gamma1=1e-4, theta_s_deg=90.0, dt=dt)


def c2_param_dict(dt=5e-5):
    eta = 0.01
    return dict(rho1=1.0, rho2=1000.0, mu1=0.01, mu2=1.0, eps1=0.025, eps2=1.0,
                lam=lam_from_sigma(1.0, eta), eta=eta, gamma1=1e-4, theta_s_deg=90.0, dt=dt)


C1 = dict(name="C1", nx=4, ny=4, K=6, steps=100, center=(0.5, 0.5), r=0.25, vtop=(1.0,))
C2 = dict(name="C2", nx=20, ny=20, K=8, steps=2000, center=(0.5, 0.0), r=0.25,
          vtop=(0.0, 0.5, 1.0, 2.0))


def c3_param_dict(dt=1e-4):
    eta = 0.02
    return dict(rho1=1.0, rho2=10.0, mu1=0.01, mu2=0.02, eps1=0.1, eps2=1.0,
                lam=lam_from_sigma(1.0, eta), eta=eta, gamma1=1e-4, theta_s_deg=90.0, dt=dt)


C3 = dict(name="C3", nx=16, ny=16, K=8, nz=128, lz=2.0, steps=500, center=(0.5, 0.5, 1.0), r=0.3,
          seed=230509020)


def perturbation(X, Y, Z, lz, seed, n=8, kmax=2):
    """xi(x) = sum_i a_i cos(2 pi (kx x + ky y + kz z / lz) + p_i), integer wave vectors in
    [-kmax, kmax]^3 (not all zero), a_i >= 0 with sum 1, phases uniform; PCG64(seed)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    ks = []
    while len(ks) < n:
        k = rng.integers(-kmax, kmax + 1, size=3)
        if np.any(k != 0):
            ks.append(k)
    a = rng.random(n)
    a = a / a.sum()
    ph = rng.random(n) * 2.0 * np.pi
    xi = np.zeros(np.broadcast(X, Y, Z).shape)
    for i in range(n):
        xi = xi + a[i] * np.cos(2.0 * np.pi * (ks[i][0] * X + ks[i][1] * Y + ks[i][2] * Z / lz) + ph[i])
    return xi


def c3_phi0(X, Y, Z):
    """Initial phase field of C3 on node coordinates (arrays of one shape)."""
    xi = perturbation(X, Y, Z, C3["lz"], C3["seed"])
    r = C3["r"] * (1.0 + 0.01 * xi)
    d = np.sqrt((X - C3["center"][0]) ** 2 + (Y - C3["center"][1]) ** 2 + (Z - C3["center"][2]) ** 2)
    return np.tanh((d - r) / (math.sqrt(2.0) * c3_param_dict()["eta"]))


# ---- batched workload: 64 independent 2D instances of uneven mesh and order
C4 = dict(name="C4", n_inst=64, seed=1, n_range=(8, 24), K_range=(4, 10), vtop=(0.0, 2.0),
          eps_ratio=(1.5, 40.0), steps=200, center=(0.5, 0.5), r=0.25)


def c4_param_dict(eps_ratio, dt=1e-4):
    """C1's fluids with eta = 0.02 and permittivities 0.1 : 0.1*eps_ratio."""
    eta = 0.02
    return dict(rho1=1.0, rho2=2.0, mu1=0.01, mu2=0.02, eps1=0.1, eps2=0.1 * eps_ratio,
                lam=lam_from_sigma(1.0, eta), eta=eta, gamma1=1e-4, theta_s_deg=90.0, dt=dt)


def c4_instances(n_inst=None, seed=None):
    """Seeded instance list: square meshes n x n with n ~ U{8..24}, order K ~ U{4..10},
    top voltage ~ U[0, 2], permittivity ratio ~ U[1.5, 40] (numpy PCG64)."""
    n_inst = C4["n_inst"] if n_inst is None else n_inst
    rng = np.random.default_rng(C4["seed"] if seed is None else seed)
    out = []
    for _ in range(n_inst):
        n = int(rng.integers(C4["n_range"][0], C4["n_range"][1] + 1))
        K = int(rng.integers(C4["K_range"][0], C4["K_range"][1] + 1))
        v = float(rng.uniform(*C4["vtop"]))
        er = float(rng.uniform(*C4["eps_ratio"]))
        out.append(dict(n=n, K=K, vtop=v, eps_ratio=er))
    return out


# ---- equilibrium workload with partial electrodes (learned warm start)
# run settings actually used (eta_run, dt_run): a resolved interface (eta 0.04 over the 1/64 z
# spacing) and the step the march stays stable at, in place of the proposed eta and dt;
# n_train_run / n_test_run: 512 training and 32 held-out problems; a training draw whose march
# has not reached the tolerance after gen_max_steps is left out of the training set (held-out
# marches run to max_steps)
C5 = dict(name="C5", nx=12, ny=12, K=6, nz=64, lx=1.0, ly=0.5, lz=1.0, center=(0.5, 0.0, 0.5),
          eta_run=0.04, dt_run=5e-5, tol=1e-8, n_train_run=512, n_test_run=32, max_steps=20000,
          gen_max_steps=5000,
          r=0.25, eta=0.02, lam_gamma1=0.1, dt=1e-5, eps1=1e-3, vrange=(0.0, 2.0), eps_ratio=(1.5, 40.0),
          theta=(60.0, 120.0), n_train=512, n_test=32, seed_train=2, seed_test=3)


def c5_electrodes(nx=None, lx=None):
    """Bottom-wall electrode segments: the x-elements cycle (+V, gap, -V, gap); returns
    [(x0, x1, sign)] for the electrode elements."""
    nx = C5["nx"] if nx is None else nx
    lx = C5["lx"] if lx is None else lx
    h = lx / nx
    out = []
    for e in range(nx):
        t = e % 4
        if t == 0:
            out.append((e * h, (e + 1) * h, 1.0))
        elif t == 2:
            out.append((e * h, (e + 1) * h, -1.0))
    return out


def c5_param_dict(eps_ratio, theta_deg, dt=None, eta=None, eps1=None):
    """Equilibrium-system parameters: eta = 0.02, lambda gamma1 = 0.1, eps1 = 1e-3 (phase 1,
    phi = +1, the ambient fluid) and eps2 = eps1 * eps_ratio (the drop, phi = -1).  The
    permittivity scale keeps eps2 V^2 <= 0.16 at the largest voltage and ratio: the oracle's
    equilibrium march diverges within a few steps from about eps2 V^2 = 0.3 whatever the step."""
    eta = C5["eta"] if eta is None else eta
    eps1 = C5["eps1"] if eps1 is None else eps1
    lam = lam_from_sigma(1.0, eta)
    return dict(rho1=1.0, rho2=1.0, mu1=0.01, mu2=0.01, eps1=eps1, eps2=eps1 * float(eps_ratio), lam=lam,
                eta=eta, gamma1=C5["lam_gamma1"] / lam, theta_s_deg=float(theta_deg),
                dt=C5["dt"] if dt is None else dt)


def c5_samples(n, seed):
    """Seeded parameter draws (V, eps ratio, contact angle), numpy PCG64."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        out.append((float(rng.uniform(*C5["vrange"])), float(rng.uniform(*C5["eps_ratio"])),
                    float(rng.uniform(*C5["theta"]))))
    return out


def c5_vd(X, Y, V, electrodes, tol=1e-12):
    """Dirichlet data on the electrode nodes of the bottom row: +V / -V by segment."""
    vd = np.zeros_like(np.asarray(X, dtype=float))
    bottom = np.isclose(Y, 0.0)
    for (x0, x1, sgn) in electrodes:
        vd = np.where(bottom & (X >= x0 - tol) & (X <= x1 + tol), sgn * V, vd)
    return vd


# ---- the paper's drop transport (Sec. 4.4.1): a dielectric drop pulled along a wall by an
# electrode array, in the normalised units of its Table 1
X6 = dict(name="X6", lx=1.6, ly=0.5, nx=16, ny=4, K=12, center=(1.2, 0.0), r=0.35, steps=2000,
          # bottom-wall electrodes (x0, x1, sign of the voltage V0); the right half is bare
          electrodes=((0.1, 0.2, -1.0), (0.3, 0.4, 1.0), (0.5, 0.6, -1.0), (0.7, 0.8, 1.0)),
          # dimensional inputs of Sec. 4.4.1 (SI units)
          L0=1e-3, V0=300.0, sigma=2.84e-2, rho=429.7, mu1=12.048e-4, eps_vac=8.854e-12,
          eps_ratio=8.1, eta=0.01, gamma1=5e-6, dt=1e-6, theta=90.0)


def x6_param_dict():
    """Normalised parameters of the drop-transport run: lengths by L0, potentials by V0,
    viscosities by mu1, permittivities by the vacuum value, densities by mu1^2/(eps V0^2),
    lambda by eps V0^2, gamma1 by L0^2/mu1, time by L0^2 mu1/(eps V0^2) (Table 1)."""
    L0, V0, mu0, e0 = X6["L0"], X6["V0"], X6["mu1"], X6["eps_vac"]
    rho_n = mu0 ** 2 / (e0 * V0 ** 2)
    lam = 3.0 / (2.0 * math.sqrt(2.0)) * X6["sigma"] * X6["eta"] * L0 / (e0 * V0 ** 2)
    return dict(rho1=X6["rho"] / rho_n, rho2=X6["rho"] / rho_n, mu1=1.0, mu2=2.0, eps1=1.0,
                eps2=X6["eps_ratio"], lam=lam, eta=X6["eta"], gamma1=X6["gamma1"],
                theta_s_deg=X6["theta"], dt=X6["dt"])


def x6_vd(X, Y, tol=1e-12):
    """Electrode voltages (+-1 in units of V0) on the electrode nodes of the bottom row."""
    vd = np.zeros_like(np.asarray(X, dtype=float))
    bottom = np.isclose(Y, 0.0)
    for (x0, x1, sgn) in X6["electrodes"]:
        vd = np.where(bottom & (X >= x0 - tol) & (X <= x1 + tol), sgn, vd)
    return vd


# ---- the paper's 3D dielectric drop on an electrode array (Sec. 4.2), equilibrium system,
# normalised as its Table 2 (lengths by L0 = 1.2 mm, potential by V0, permittivities by
# L0 sigma / V0^2); the contact angle is not stated there: 90 deg (the initial hemisphere)
X3 = dict(name="X3", lx=5.0 / 3.0, ly=2.0 / 3.0, lz=3.5, nx=20, ny=6, K=12, nz=120,
          # six elements along y, finer at the wall where the drop and the field gradients sit
          yb=(0.0, 0.04, 0.1, 0.18, 0.3, 0.46, 2.0 / 3.0),
          center=(5.0 / 6.0, 0.0, 1.75), r=0.5, eta=0.02, lam_gamma1=0.1, dt=2e-6,
          L0=1.2e-3, sigma=3.857e-2, eps_vac=8.854e-12, eps_ratio=32.0, V0=150.0, theta=90.0, steps=200)


def x3_param_dict(V0=None):
    """Equilibrium-system parameters of the 3D drop: eps1 = eps_vac V0^2 / (L0 sigma),
    eps2 = 32 eps1, lambda = 3 sigma eta / (2 sqrt 2) with sigma = 1, lambda gamma1 = 0.1."""
    V0 = X3["V0"] if V0 is None else V0
    e1 = X3["eps_vac"] * V0 ** 2 / (X3["L0"] * X3["sigma"])
    lam = lam_from_sigma(1.0, X3["eta"])
    return dict(rho1=1.0, rho2=1.0, mu1=0.01, mu2=0.01, eps1=e1, eps2=X3["eps_ratio"] * e1, lam=lam,
                eta=X3["eta"], gamma1=X3["lam_gamma1"] / lam, theta_s_deg=X3["theta"], dt=X3["dt"])


def x3_electrodes():
    """The x-elements alternate electrode / gap (width L0/12 each, 20 elements over 5/3):
    electrodes on the even elements, voltages alternating +1, -1; [(x0, x1, sign)]."""
    h = X3["lx"] / X3["nx"]
    out = []
    for e in range(0, X3["nx"], 2):
        out.append((e * h, (e + 1) * h, 1.0 if (e // 2) % 2 == 0 else -1.0))
    return out


def electrode_vd(X, Y, electrodes, tol=1e-12):
    """Dirichlet data on the electrode nodes of the bottom row: sign * 1 by segment."""
    vd = np.zeros_like(np.asarray(X, dtype=float))
    bottom = np.isclose(Y, 0.0)
    for (x0, x1, sgn) in electrodes:
        vd = np.where(bottom & (X >= x0 - tol) & (X <= x1 + tol), sgn, vd)
    return vd


# ---- the paper's 2D dielectric film (Sec. 4.3), equilibrium system, normalised with
# L0 = d/2 (so the domain is [0,8] x [0,5]) and Vd = 100 V; electrodes on x in [1,3]
# (V = 0) and [5,7] (V = V0); the film thickness h0, its permittivity, the electrode width
# and the element counts along x are not fixed there (proposals here)
X4 = dict(name="X4", lx=8.0, ly=5.0, nx=16, K=12, h0=1.0, amp=0.2, ny_regions=(5, 4, 4),
          electrodes=((1.0, 3.0, 0.0), (5.0, 7.0, 1.0)), eta=0.01, lam_gamma1=0.1, dt=2e-6,
          d=1e-4, Vd=100.0, sigma=2.84e-2, eps_vac=8.854e-12, eps_ratio=10.0, theta=90.0, steps=500)


def x4_mesh_y():
    """y breakpoints: near-wall region [0, h0 - A/2] and wave region [h0 - A/2, h0 + A/2] with
    uniform elements, the upper region up to 5 with elements growing by 1.6."""
    n1, n2, n3 = X4["ny_regions"]
    a, b = X4["h0"] - X4["amp"] / 2, X4["h0"] + X4["amp"] / 2
    ys = list(np.linspace(0.0, a, n1 + 1)) + list(np.linspace(a, b, n2 + 1))[1:]
    g = 1.6 ** np.arange(n3)
    ys += list(b + (X4["ly"] - b) * np.cumsum(g) / g.sum())
    return np.array(ys)


def x4_param_dict():
    """Equilibrium-system parameters of the film.  The stabiliser is set to S = 2: the paper
    only bounds S from below, by the value that splits the Cahn-Hilliard step into two
    Helmholtz problems (0.548 here), and at that value the march diverges (the oracle's too,
    at any voltage); the linear stabilisation of the double well needs S of the order of
    max h'(phi) eta^2 = 2 (S = 1 still diverged, S = 2 marched stably at V0 = 1 and 3)."""
    L0 = X4["d"] / 2.0
    e1 = X4["eps_vac"] * X4["Vd"] ** 2 / (L0 * X4["sigma"])
    lam = lam_from_sigma(1.0, X4["eta"])
    return dict(rho1=1.0, rho2=1.0, mu1=0.01, mu2=0.01, eps1=e1, eps2=X4["eps_ratio"] * e1, lam=lam,
                eta=X4["eta"], gamma1=X4["lam_gamma1"] / lam, theta_s_deg=X4["theta"], dt=X4["dt"], S=2.0)


def x4_phi0(Y):
    """Flat film of thickness h0: phi = tanh((y - h0) / (sqrt 2 eta)) (film phi = -1)."""
    return np.tanh((np.asarray(Y) - X4["h0"]) / (math.sqrt(2.0) * X4["eta"]))
