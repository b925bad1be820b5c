"""Sampled oracle fields of the 3D benchmark workload at full size (oracle only).

Workload: [0,1]^2 x [0,2) (z periodic), 16x16 elements of order 8, 128 Fourier planes
(129 x 129 x 128 = 2,130,048 nodes), the perturbed sphere of the synth module's C3 settings,
walls, V = 0 at the bottom and 1 at the top, dt = 1e-4.  Initial potential V = y (the
Dirichlet data extended linearly; the test sets the same on the GPU, so the fixed point of
Remark 3.1 is not needed).  The oracle (Algorithm 2, eqs. 74-78, per-mode sparse LU) takes
two steps; the fields phi, psi, V, P, u_x, u_y, u_z are stored after each at 4096 nodes
drawn with a seeded generator, with each field's maximum over all nodes.

Usage: python tests/golden/make_c3_sample.py   (a few minutes)
Output: tests/golden/c3_sample.npz
"""
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

from oracle.sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT  # noqa: E402
from oracle.scheme import Scheme, Params, BCs, WALL  # noqa: E402
from synth import C3, c3_param_dict, c3_phi0  # noqa: E402

FIELDS = ("phi", "psi", "V", "P", "ux", "uy", "uz")
NSAMPLE = 4096


def main():
    par = Params(**c3_param_dict())
    xb = np.linspace(0.0, 1.0, C3["nx"] + 1)
    m = Mesh2D(xb, xb, C3["K"])
    bc = BCs(side={BOTTOM: WALL, TOP: WALL, LEFT: WALL, RIGHT: WALL}, pot_sides=(BOTTOM, TOP))
    sch = Scheme(m, par, bc, Nz=C3["nz"], Lz=C3["lz"], lu_order="MMD_AT_PLUS_A")   # fast factorisations
    Z = np.broadcast_to(sch.z[:, None], (C3["nz"], m.Ng))
    X = np.broadcast_to(m.X.ravel()[None, :], Z.shape)
    Y = np.broadcast_to(m.Y.ravel()[None, :], Z.shape)
    sch.set_state(c3_phi0(X, Y, Z))
    sch.state["cur"]["V"] = np.array(Y)
    sch.state["old"]["V"] = np.array(Y)
    src = dict(Vd=np.where(np.isclose(Y, 1.0), 1.0, 0.0))
    rng = np.random.default_rng(3051)
    idx = rng.choice(C3["nz"] * m.Ng, size=NSAMPLE, replace=False)
    arrays = dict(index=idx)
    for n in (1, 2):
        o = sch.step(src)
        for k in FIELDS:
            f = np.asarray(o[k]).ravel()
            arrays["%s_%d" % (k, n)] = f[idx]
            arrays["max_%s_%d" % (k, n)] = np.array(np.abs(f).max())
        print("step", n, flush=True)
    path = os.path.join(HERE, "c3_sample.npz")
    np.savez_compressed(path, **arrays)
    print("wrote", path)


if __name__ == "__main__":
    main()
