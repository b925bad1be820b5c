"""Build C-ABI contexts that mirror the oracle test cases (same mesh, parameters,
boundary conditions and input arrays)."""
import numpy as np

from oracle.sem import BOTTOM, TOP, LEFT, RIGHT
from oracle.scheme import WALL, OPEN


def params_dict(par):
    return dict(rho1=par.rho1, rho2=par.rho2, mu1=par.mu1, mu2=par.mu2, eps1=par.eps1,
                eps2=par.eps2, lam=par.lam, eta=par.eta, gamma1=par.gamma1,
                theta_s_deg=par.theta_s_deg, dt=par.dt, bdf=par.bdf, S=par.S, nu_m=par.nu_m)


def gpu_context(mesh, par, bc, nbatch=1, precision=0, refine_max=0, nz=0, lz=0.0, refine_tol=0.0):
    import paper_2305_09020_amd as pfd
    st = [pfd.WALL] * 4
    for s, typ in bc.side.items():
        st[s] = pfd.WALL if typ == WALL else pfd.OPEN
    pdir = [1 if s in bc.pot_sides else 0 for s in range(4)]
    prob = pfd.make_problem(mesh.xb, mesh.yb, mesh.K, params_dict(par), st, pdir,
                            periodic_x=mesh.periodic_x, nbatch=nbatch, nz=nz, lz=lz, precision=precision,
                            refine_max=refine_max, refine_tol=refine_tol,
                            electrodes=bc.electrodes)
    return pfd.Context(prob)


def rel_err(a, b):
    a = np.asarray(a).ravel()
    b = np.asarray(b).ravel()
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)
