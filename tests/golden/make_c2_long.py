"""Write the long-run fixtures of the 2D benchmark workload from the FP64 oracle only.

Workload: [0,1]^2, 20x20 elements of order 8, sessile half-disc r = 0.25 at (0.5, 0),
eta = 0.01, rho 1:1000, mu 0.01:1, eps 0.025:1, closed box, V = 0 at the bottom and
V_top = 2 at the top, dt = 5e-5 (the synth module's C2 settings, instance V_top = 2).
The oracle (Algorithm 1, eqs. 54-59, sparse LU) is stepped 2000 times from the initial
potential of Remark 3.1 (stored as V_0); phi, psi, V, P, u_x, u_y are stored after steps 1,
10, 100 and 2000.

Rounding floors, stored beside the fields as the per-field max |a - b| / max |a| at each
checkpoint:
  sens_*  the same run from phi0 perturbed node by node by one unit in the last place (a
          seeded random sign per node): how much the workload amplifies a rounding-level
          change of its input;
  twin_*  the same run with a second column ordering of the sparse LU factorisations
          (MMD on A^T + A instead of COLAMD): a second, equally valid FP64 rounding of every
          step of the same scheme.  Two correct FP64 implementations that round differently
          cannot be expected to agree more closely than this.

Usage: python tests/golden/make_c2_long.py  (about 8 minutes; three processes)
Output: tests/golden/c2_vtop2_long.npz
"""
import os
import sys
import time
from multiprocessing import Pool

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT  # noqa: E402
from oracle.scheme import Scheme, Params, BCs, WALL  # noqa: E402
from synth import C2, c2_param_dict, drop_field  # noqa: E402

CHECKPOINTS = (1, 10, 100, 2000)
FIELDS = ("phi", "psi", "V", "P", "ux", "uy")
VTOP = 2.0


def workload():
    par = Params(**c2_param_dict())
    xb = np.linspace(0.0, 1.0, C2["nx"] + 1)
    m = Mesh2D(xb, xb, C2["K"])
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    phi0 = drop_field(m.X, m.Y, C2["center"], C2["r"], par.eta).ravel()
    vd = np.where(np.isclose(m.Y.ravel(), 1.0), VTOP, 0.0)
    return par, m, bc, phi0, vd


def run(kind):
    par, m, bc, phi0, vd = workload()
    if kind == "perturbed":
        rng = np.random.default_rng(2305)
        phi0 = phi0 + np.spacing(phi0) * rng.choice([-1.0, 1.0], size=phi0.shape)
    sch = Scheme(m, par, bc, lu_order="MMD_AT_PLUS_A" if kind == "twin" else "COLAMD")
    sch.set_state(phi0)
    src = dict(Vd=vd)
    V0 = sch.init_potential(src)[0].reshape(m.Ny, m.Nx).copy()
    out = {0: dict(V=V0)}
    t0 = time.perf_counter()
    for n in range(1, CHECKPOINTS[-1] + 1):
        o = sch.step(src)
        if n in CHECKPOINTS:
            out[n] = {k: np.array(o[k]).reshape(m.Ny, m.Nx) for k in FIELDS}
            print("%s step %d (%.0f s)" % (kind, n, time.perf_counter() - t0), flush=True)
    return out


def main():
    with Pool(3) as pool:
        base, pert, twin = pool.map(run, ["base", "perturbed", "twin"])
    arrays = {}
    for n in CHECKPOINTS:
        for k in FIELDS:
            a = base[n][k]
            arrays["%s_%d" % (k, n)] = a
            for tag, other in (("sens", pert), ("twin", twin)):
                b = other[n][k]
                arrays["%s_%s_%d" % (tag, k, n)] = np.array(np.abs(a - b).max() / max(np.abs(a).max(), 1e-300))
    arrays["checkpoints"] = np.array(CHECKPOINTS)
    arrays["V_0"] = base[0]["V"]   # the initial potential (Remark 3.1, solved directly)
    path = os.path.join(HERE, "c2_vtop2_long.npz")
    np.savez_compressed(path, **arrays)
    for tag in ("sens", "twin"):
        for n in CHECKPOINTS:
            print("%s after %4d steps: " % (tag, n) +
                  " ".join("%s %.2e" % (k, float(arrays["%s_%s_%d" % (tag, k, n)])) for k in FIELDS))
    print("wrote", path)


if __name__ == "__main__":
    main()
