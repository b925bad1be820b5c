"""Manufactured solutions of Sec. 4.1 (eq. 80 in 2D, eq. 81 in 3D) and the source
terms that make them exact solutions of the source-augmented system
(eqs. 27-33 of Sec. 3.1: g, f, f_V, g1, g2, g3, f1, f2, w).

The sources are derived symbolically (SymPy) from the continuous equations:
  g   = phi_t + u.grad phi - gamma1 lap(mu_c),
        mu_c = lambda h(phi) - lambda lap phi - eps'(phi)/2 |grad V|^2      (eqs. 6, ecp)
  f   = rho (u_t + u.grad u) + J~.grad u + lambda lap phi grad phi
        + eps'/2 |E|^2 grad phi - mu lap u - grad mu . D(u) + grad P,
        J~ = -gamma1 (rho1-rho2)/2 grad mu_c                                (eq. 28)
  f_V = div(eps(phi) grad V)                                                (eq. 28)
  g1  = n.grad[lap phi - h(phi) + eps'(phi)|E|^2/(2 lambda)]  (scheme's eq. phia)
  g2  = n.grad phi (open),  g3 = -n.grad phi - Theta'(phi)/lambda (eq. phic)
  f1  = du/dn (open),  f2 = P (open),  w = u (wall),  V = V_exact on Dirichlet nodes.
"""
import functools
import math

import numpy as np
import sympy as s

X, Y, Z, T = s.symbols("x y z t", real=True)


def exact_2d():
    """eq. (80)."""
    pi = s.pi
    u = s.cos(pi * Y) * s.sin(pi * X) * s.sin(T)
    v = -s.sin(pi * Y) * s.cos(pi * X) * s.sin(T)
    P = s.sin(pi * Y) * s.cos(pi * X) * s.cos(T)
    phi = s.cos(pi * X) * s.cos(pi * Y) * s.sin(T)
    V = s.sin(pi * X) * s.cos(pi * Y)
    return dict(u=(u, v, s.Integer(0)), P=P, phi=phi, V=V)


def exact_3d():
    """eq. (81)."""
    pi = s.pi
    u = s.cos(pi * X) * s.cos(pi * Y) * s.cos(pi * Z) * s.sin(T)
    v = s.Integer(0)
    w = s.sin(pi * X) * s.cos(pi * Y) * s.sin(pi * Z) * s.sin(T)
    P = s.sin(pi * X) * s.sin(pi * Y) * s.sin(pi * Z) * s.cos(T)
    phi = s.cos(pi * X) * s.cos(pi * Y) * s.cos(pi * Z) * s.sin(T)
    V = s.sin(pi * X) * s.cos(pi * Y) * s.cos(pi * Z)
    return dict(u=(u, v, w), P=P, phi=phi, V=V)


def exact_box():
    """A closed-box solution on [0,1]^2 (not from the paper; it exercises the
    wall-only configuration): no-slip walls from the stream function
    sin^2(pi x) sin^2(pi y) sin t, dphi/dn = 0 and n.grad mu_c = 0 on every wall,
    V = 0 at y = 0, V = 1 at y = 1 and dV/dn = 0 on x = 0, 1."""
    pi = s.pi
    sf = s.sin(pi * X) ** 2 * s.sin(pi * Y) ** 2 * s.sin(T)
    u = s.diff(sf, Y)
    v = -s.diff(sf, X)
    P = s.cos(pi * X) * s.cos(pi * Y) * s.cos(T)
    phi = s.Rational(1, 2) * s.cos(pi * X) * s.cos(pi * Y) * s.sin(T)
    V = Y + s.Rational(1, 10) * s.sin(pi * Y) * s.cos(pi * X)
    return dict(u=(u, v, s.Integer(0)), P=P, phi=phi, V=V)


def exact_slab():
    """A 3D solution between no-slip walls at y = -1 and y = 1 (not from the paper;
    it exercises the 3D terms without tangential wall motion): u = curl(b, 0, a)
    with a = sin^2(pi y) cos(pi x) cos(pi z) sin t and
    b = sin^2(pi y) sin(pi x) sin(pi z) sin t, so div u = 0 and u = 0 on both walls,
    and every component varies along z."""
    pi = s.pi
    a = s.sin(pi * Y) ** 2 * s.cos(pi * X) * s.cos(pi * Z) * s.sin(T)
    b = s.sin(pi * Y) ** 2 * s.sin(pi * X) * s.sin(pi * Z) * s.sin(T)
    u = s.diff(a, Y)
    v = -s.diff(a, X) + s.diff(b, Z)
    w = -s.diff(b, Y)
    P = s.cos(pi * X) * s.cos(pi * Y) * s.sin(pi * Z) * s.cos(T)
    phi = s.Rational(1, 2) * s.cos(pi * X) * s.cos(pi * Y) * s.cos(pi * Z) * s.sin(T)
    V = s.sin(pi * X) * s.cos(pi * Y) * s.cos(pi * Z)
    return dict(u=(u, v, w), P=P, phi=phi, V=V)


EXACT = {"eq80": (2, exact_2d), "eq81": (3, exact_3d), "box": (2, exact_box),
         "slab": (3, exact_slab)}


def _grad(f):
    return [s.diff(f, X), s.diff(f, Y), s.diff(f, Z)]


def _lap(f):
    return s.diff(f, X, 2) + s.diff(f, Y, 2) + s.diff(f, Z, 2)


@functools.lru_cache(maxsize=8)
def _sources(kind, rho1, rho2, mu1, mu2, eps1, eps2, lam, eta, gamma1, theta):
    ex = EXACT[kind][1]()
    u = list(ex["u"])
    P, phi, V = ex["P"], ex["phi"], ex["V"]
    rho = (rho1 + rho2) / 2 + (rho1 - rho2) / 2 * phi
    mu = (mu1 + mu2) / 2 + (mu1 - mu2) / 2 * phi
    eps = (eps1 + eps2) / 2 + (eps1 - eps2) / 2 * phi * (3 - phi ** 2) / 2
    deps = (eps2 - eps1) / 2 * 3 * (phi ** 2 - 1) / 2
    h = phi * (phi ** 2 - 1) / eta ** 2
    E = _grad(V)
    E2 = sum(e * e for e in E)
    muc = lam * h - lam * _lap(phi) - deps / 2 * E2
    gphi = _grad(phi)
    g = s.diff(phi, T) + sum(u[i] * gphi[i] for i in range(3)) - gamma1 * _lap(muc)
    Jt = [-gamma1 * (rho1 - rho2) / 2 * d for d in _grad(muc)]
    gu = [_grad(uk) for uk in u]          # gu[k][i] = d_i u_k
    gmu = _grad(mu)
    gP = _grad(P)
    f = []
    for k in range(3):
        adv = sum(u[i] * gu[k][i] for i in range(3))
        jdu = sum(Jt[i] * gu[k][i] for i in range(3))
        gmD = sum(gmu[i] * (gu[k][i] + gu[i][k]) for i in range(3))
        f.append(rho * (s.diff(u[k], T) + adv) + jdu + lam * _lap(phi) * gphi[k]
                 + deps / 2 * E2 * gphi[k] - mu * _lap(u[k]) - gmD + gP[k])
    fV = sum(s.diff(eps * E[i], v) for i, v in enumerate((X, Y, Z)))
    bq = _lap(phi) - h + deps * E2 / (2 * lam)
    gbq = _grad(bq)
    thp = math.cos(math.radians(theta)) * (phi ** 2 - 1) / (math.sqrt(2) * eta)
    out = dict(g=g, fx=f[0], fy=f[1], fz=f[2], fV=fV, V=V, P=P, phi=phi,
               ux=u[0], uy=u[1], uz=u[2])
    # boundary pieces: normal derivatives along x and y
    out["_g1"] = [gbq[0], gbq[1]]
    out["_gphi"] = [gphi[0], gphi[1]]
    out["_thp"] = thp
    out["_dux"] = [s.diff(u[k], X) for k in range(3)]
    out["_duy"] = [s.diff(u[k], Y) for k in range(3)]
    args = (X, Y, Z, T)
    num = {}
    for k, v in out.items():
        if isinstance(v, list):
            num[k] = [s.lambdify(args, e, "numpy") for e in v]
        else:
            num[k] = s.lambdify(args, v, "numpy")
    return num


def _ev(fn, x, y, z, t):
    r = fn(x, y, z, t)
    return np.broadcast_to(np.asarray(r, dtype=np.float64), np.broadcast(x, y, z).shape).copy()


class Manufactured:
    """Evaluate the exact fields and sources on given node coordinates.

    kind: "eq80" (2D, eq. 80), "eq81" (3D, eq. 81), "box" (2D closed box) or
    "slab" (3D between two no-slip walls).
    Boundary sources are nodal; the side of each boundary node is given by masks.
    A node on two sides (a corner) takes the value of the side listed last; the
    "box" solution has zero normal-derivative data on every side, so its
    corners are unambiguous.
    """

    def __init__(self, kind, par):
        self.kind = kind
        self.dim = EXACT[kind][0]
        self.par = par
        self.fn = _sources(kind, par.rho1, par.rho2, par.mu1, par.mu2, par.eps1, par.eps2,
                           par.lam, par.eta, par.gamma1, par.theta_s_deg)

    def fields(self, x, y, z, t):
        F = self.fn
        return dict(phi=_ev(F["phi"], x, y, z, t), P=_ev(F["P"], x, y, z, t),
                    V=_ev(F["V"], x, y, z, t),
                    u=(_ev(F["ux"], x, y, z, t), _ev(F["uy"], x, y, z, t),
                       _ev(F["uz"], x, y, z, t)))

    def sources(self, x, y, z, t, sides):
        """Nodal source arrays at time t.

        sides: list of (mask, (nx, ny), type) with type "wall" or "open"; boundary
        sources are zero away from these masks."""
        F = self.fn
        src = {k: _ev(F[k], x, y, z, t) for k in ("g", "fx", "fy", "fz", "fV")}
        zero = np.zeros(np.broadcast(x, y, z).shape)
        for k in ("g1", "g2", "g3", "f1x", "f1y", "f1z", "f2", "wx", "wy", "wz"):
            src[k] = zero.copy()
        src["Vd"] = _ev(F["V"], x, y, z, t)
        g1 = [_ev(f, x, y, z, t) for f in F["_g1"]]
        gp = [_ev(f, x, y, z, t) for f in F["_gphi"]]
        th = _ev(F["_thp"], x, y, z, t)
        du = ([_ev(f, x, y, z, t) for f in F["_dux"]], [_ev(f, x, y, z, t) for f in F["_duy"]])
        uex = [_ev(F[k], x, y, z, t) for k in ("ux", "uy", "uz")]
        pex = _ev(F["P"], x, y, z, t)
        for mask, (nx, ny), typ in sides:
            src["g1"][mask] = (nx * g1[0] + ny * g1[1])[mask]
            dn = nx * gp[0] + ny * gp[1]
            if typ == "open":
                src["g2"][mask] = dn[mask]
                for k, name in enumerate(("f1x", "f1y", "f1z")):
                    src[name][mask] = (nx * du[0][k] + ny * du[1][k])[mask]
                src["f2"][mask] = pex[mask]
            else:
                src["g3"][mask] = (-dn - th)[mask]
                for k, name in enumerate(("wx", "wy", "wz")):
                    src[name][mask] = uex[k][mask]
        return src
