"""Shared test cases: manufactured-solution setups of Sec. 4.1 and small
physical setups, described once and run through the oracle (and, in the GPU
tests, through the C-ABI library with the same input arrays)."""
import numpy as np

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT, NORMALS
from oracle.scheme import Scheme, Params, BCs, WALL, OPEN
from oracle.manufactured import Manufactured
from synth import c1_param_dict, c2_param_dict


def c1_params(dt=1e-4):
    return Params(**c1_param_dict(dt))


def c2_params(dt=5e-5):
    return Params(**c2_param_dict(dt))


def mms_params(dt=1e-3, S=0.0):
    # the paper does not state the physical parameters of its convergence tests;
    # these are moderate values with every property contrast switched on
    return Params(rho1=1.0, rho2=3.0, mu1=0.01, mu2=0.02, eps1=1.0, eps2=4.0, lam=0.01,
                  eta=0.1, gamma1=0.01, theta_s_deg=75.0, dt=dt, S=S)


def mms_setup(kind, K, dt, Nz=8, S=0.0, par=None):
    """Mesh, BCs and side masks of the manufactured tests.

    eq80: [0,2]x[0,1], two elements, x-periodic, wall at y=0 (V Dirichlet), open top.
    eq81: [0,2]x[-1,1]x[0,2], two elements split at x=1, Nz planes, V Dirichlet on
          x in [0,1] of the bottom wall, Neumann on x in [1,2].
    eq81b: eq81 with V Dirichlet on the whole bottom wall.
    eq81w: eq81 with walls at y=-1 and y=1 (V Dirichlet on both), no open boundary.
    slab: the eq81w domain and sides on 4x4 elements, with a solution that vanishes on
          both walls.
    box:  [0,1]^2, 2x2 elements, walls everywhere, V Dirichlet at y=0 and y=1.
    """
    par = par or mms_params(dt, S)
    if kind == "eq80":
        m = Mesh2D([0.0, 1.0, 2.0], [0.0, 1.0], K, periodic_x=True)
        bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, pot_sides=(BOTTOM,))
        sch = Scheme(m, par, bc)
    elif kind in ("eq81", "eq81b", "eq81w", "slab"):
        if kind == "slab":
            m = Mesh2D([0.0, 0.5, 1.0, 1.5, 2.0], [-1.0, -0.5, 0.0, 0.5, 1.0], K,
                       periodic_x=True)
        else:
            m = Mesh2D([0.0, 1.0, 2.0], [-1.0, 1.0], K, periodic_x=True)
        if kind == "eq81":
            bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, electrodes=[(0.0, 1.0)])
        elif kind == "eq81b":  # same solution with V Dirichlet on the whole bottom wall
            bc = BCs(side={BOTTOM: WALL, TOP: OPEN}, pot_sides=(BOTTOM,))
        else:  # two walls (no open boundary), V Dirichlet on both
            bc = BCs(side={BOTTOM: WALL, TOP: WALL}, pot_sides=(BOTTOM, TOP))
        sch = Scheme(m, par, bc, Nz=Nz, Lz=2.0)
    elif kind == "box":
        m = Mesh2D([0.0, 0.5, 1.0], [0.0, 0.5, 1.0], K, periodic_x=False)
        bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL},
                 pot_sides=(BOTTOM, TOP))
        sch = Scheme(m, par, bc)
    else:
        raise ValueError(kind)
    Nzz = sch.Nz
    x = np.broadcast_to(m.X.ravel()[None, :], (Nzz, m.Ng)).copy()
    y = np.broadcast_to(m.Y.ravel()[None, :], (Nzz, m.Ng)).copy()
    z = (np.broadcast_to(sch.z[:, None], (Nzz, m.Ng)).copy() if sch.is3d
         else np.zeros_like(x))
    sides = []
    for s in m.sides:
        g = np.zeros(m.Ng, dtype=bool)
        g[m.side_nodes(s)] = True
        mask = np.broadcast_to(g[None, :], (Nzz, m.Ng)).copy()
        sides.append((mask, NORMALS[s], bc.side[s]))
    mf = Manufactured("eq81" if kind in ("eq81b", "eq81w") else kind, par)
    return dict(mesh=m, bc=bc, sch=sch, par=par, x=x, y=y, z=z, sides=sides, mf=mf)


def mms_initial(case, dt):
    mf = case["mf"]
    x, y, z = case["x"], case["y"], case["z"]
    return mf.fields(x, y, z, 0.0), mf.fields(x, y, z, -dt)


def mms_run_oracle(case, nsteps, dt):
    sch, mf = case["sch"], case["mf"]
    x, y, z = case["x"], case["y"], case["z"]
    f0, fm = mms_initial(case, dt)
    nc = 3 if sch.is3d else 2
    sch.set_state(f0["phi"], f0["u"][:nc], f0["P"], f0["V"],
                  prev=dict(phi=fm["phi"], u=fm["u"][:nc], P=fm["P"], V=fm["V"]))
    out = None
    for i in range(nsteps):
        out = sch.step(mf.sources(x, y, z, (i + 1) * dt, case["sides"]))
    return out


def mms_errors(case, out, t):
    fe = case["mf"].fields(case["x"], case["y"], case["z"], t)
    e = dict(phi=np.max(np.abs(out["phi"] - fe["phi"])),
             V=np.max(np.abs(out["V"] - fe["V"])),
             P=np.max(np.abs(out["P"] - fe["P"])),
             ux=np.max(np.abs(out["ux"] - fe["u"][0])),
             uy=np.max(np.abs(out["uy"] - fe["u"][1])))
    if case["sch"].is3d:
        e["uz"] = np.max(np.abs(out["uz"] - fe["u"][2]))
    return e
