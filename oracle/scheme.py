"""The decoupled time step of Sec. 3 in plain FP64 (test infrastructure only).

Paper passages followed:
  * mixture laws, eq. (interpolation); h(phi) and lambda, eq. (double_well);
  * the semi-discrete scheme eqs. (ep)-(vb), BDF-J / extrapolation (Sec. 3.1);
  * algorithmic constants eps_0 = max(eps1, eps2), rho_0 = min(rho1, rho2),
    nu_m, the stabiliser S and alpha (Sec. 3.1 and eq. 44);
  * 2D weak forms eqs. (54)-(59), Algorithm 1;
  * 3D per-Fourier-mode weak forms eqs. (74)-(78), Algorithm 2;
  * the initial potential fixed point (Remark 3.1);
  * the equilibrium ("simpler") system, eqs. (15c)-(15d) with (16).

Readings where the paper is silent, ambiguous or inconsistent (each is listed
with its reason in the design notes of the repository):
  R-basis   GLL Lagrange basis, GLL collocation quadrature (diagonal mass).
  R-bdf     BDF2 from the first step, with xi^{-1} = xi^0 unless supplied.
  R-S       S at its lower bound, radicand of alpha clamped at 0
            (so c_psi = alpha + S/eta^2 and c_phi = -alpha coincide).
  R-num     nu_m = max(mu1, mu2) / min(rho1, rho2).
  R-psi     the phi equation carries -int psi w (eq. 57); eqs. (69)/(76)
            print +int psi w, which contradicts grad^2 phi + alpha phi = psi.
  R-Ez      E_z,k = +i beta_k V_k (E = grad V, d/dz e^{i beta z} = i beta e^{i beta z});
            eqs. (70)/(78) print -i beta_k.
  R-Pbnd    the (mu/rho) n x omega* . grad q boundary integral of the pressure
            equation is taken over all of the boundary in 2D and 3D (eqs. 48, 58);
            the 3D eq. (77) prints it over the open boundary only, where q = 0.
  R-g1      g1 and g3 follow the scheme's own boundary conditions (eqs. phia,
            phic): n.grad[lap phi - h + eps'|E|^2/(2 lambda)] = g1 and
            -n.grad phi - Theta'(phi)/lambda = g3.
  R-clamp   rho and mu are evaluated at clamp(phi, -1, 1); their gradients use
            grad phi (the mixture laws are linear); eps, eps' are not clamped.
  R-Theta   Theta'(phi)/lambda = cos(theta_s)(phi^2 - 1)/(sqrt(2) eta), from
            eq. (theta_def) with lambda = 3 sigma eta / (2 sqrt 2).
  R-J       J~^{n+1} uses lap phi^{n+1} = psi - alpha phi (eq. 44b), so
            J~ = (rho1-rho2)/2 lambda gamma1 grad(psi - c_psi phi - Q2).
  R-gauge   a pressure problem with no Dirichlet boundary (closed box, or the
            k = 0 mode) is solved with its right side projected onto the range
            and the gauge int_h P = 0.
  R-nyq     modes k = 0..Nz/2; at the Nyquist mode the first-derivative factor
            i beta is set to 0 while beta^2 keeps (pi Nz / Lz)^2.
  R-dir3d   per-mode Dirichlet data is the Fourier transform of the physical
            boundary values (eq. 74b assumes z-constant electrode voltages).
  R-V0      the fixed point of Remark 3.1 is the variable-coefficient problem
            int eps(phi0) grad V . grad e = -int f_V e; the oracle solves it directly.
"""
import math
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from .sem import Mesh2D, BOTTOM, TOP, LEFT, RIGHT, NORMALS

WALL, OPEN, PERIODIC = "wall", "open", "periodic"


@dataclass
class Params:
    rho1: float
    rho2: float
    mu1: float
    mu2: float
    eps1: float
    eps2: float
    lam: float
    eta: float
    gamma1: float
    theta_s_deg: float
    dt: float
    bdf: int = 2
    S: float = 0.0          # 0 -> lower bound of Sec. 3.1 (reading R-S)
    nu_m: float = 0.0       # 0 -> max mu / min rho (reading R-num)

    def derived(self):
        """Algorithmic constants of Sec. 3.1 and eq. (44)."""
        g0 = 1.0 if self.bdf == 1 else 1.5
        lg = self.lam * self.gamma1
        Smin = self.eta ** 2 * math.sqrt(4.0 * g0 / (lg * self.dt))
        S = self.S if self.S > 0 else Smin
        rad = max(0.0, 1.0 - 4.0 * g0 / (lg * self.dt) * self.eta ** 4 / S ** 2)
        alpha = -S / (2.0 * self.eta ** 2) * (1.0 + math.sqrt(rad))
        nu_m = self.nu_m if self.nu_m > 0 else max(self.mu1, self.mu2) / min(self.rho1, self.rho2)
        return dict(
            gamma0=g0, S=S, alpha=alpha,
            c_psi=alpha + S / self.eta ** 2, c_phi=-alpha,
            eps0=max(self.eps1, self.eps2), rho0=min(self.rho1, self.rho2),
            nu_m=nu_m, c_u=g0 / (nu_m * self.dt),
        )

    # mixture laws, eq. (interpolation), and h(phi), eq. (double_well)
    def rho(self, p):
        return 0.5 * (self.rho1 + self.rho2) + 0.5 * (self.rho1 - self.rho2) * p

    def mu(self, p):
        return 0.5 * (self.mu1 + self.mu2) + 0.5 * (self.mu1 - self.mu2) * p

    def eps(self, p):
        return 0.5 * (self.eps1 + self.eps2) + 0.5 * (self.eps1 - self.eps2) * p * (3.0 - p * p) / 2.0

    def deps(self, p):
        return 0.5 * (self.eps2 - self.eps1) * 3.0 * (p * p - 1.0) / 2.0

    def h(self, p):
        return p * (p * p - 1.0) / self.eta ** 2

    def theta_p_over_lam(self, p):
        """Theta'(phi)/lambda (reading R-Theta)."""
        return math.cos(math.radians(self.theta_s_deg)) * (p * p - 1.0) / (math.sqrt(2.0) * self.eta)


@dataclass
class BCs:
    """Boundary description.

    side: type per side id (BOTTOM, TOP, LEFT, RIGHT) -> WALL | OPEN; left/right
          are omitted when the mesh is x-periodic.
    pot_sides: sides on which V is Dirichlet in full (electrode covering the side).
    electrodes: list of (x0, x1) closed segments on the bottom wall where V is
          Dirichlet (segments end on element edges).
    """
    side: dict
    pot_sides: tuple = ()
    electrodes: list = field(default_factory=list)


SRC_NAMES = ("g", "fx", "fy", "fz", "fV", "g1", "g2", "g3", "f1x", "f1y", "f1z", "f2",
             "wx", "wy", "wz", "Vd")


class Scheme:
    """One run of the decoupled scheme on a tensor mesh (2D) or mesh x Fourier (3D).

    Fields are stored as (Nz, Ng) arrays in physical space (Nz = 1 in 2D).
    Sources passed to step() are nodal arrays at t^{n+1} (missing -> 0).
    """

    def __init__(self, mesh: Mesh2D, par: Params, bc: BCs, Nz=None, Lz=None, lu_order="COLAMD"):
        # lu_order: column ordering of SuperLU (any ordering solves the same systems exactly;
        # a second ordering gives a second, equally valid rounding of the same scheme)
        self.m, self.par, self.bc = mesh, par, bc
        self.c = par.derived()
        self.is3d = Nz is not None
        self.Nz = Nz if self.is3d else 1
        self.Lz = Lz
        if self.is3d:
            if Nz < 2 or Nz % 2:
                raise ValueError("Nz must be even")
            k = np.arange(Nz // 2 + 1)
            self.beta = 2.0 * np.pi * k / Lz
            self.beta_d = self.beta.copy()
            self.beta_d[-1] = 0.0  # reading R-nyq
            self.z = np.arange(Nz) * Lz / Nz
        else:
            self.beta = np.zeros(1)
            self.beta_d = np.zeros(1)
        m = mesh
        self.open_sides = [s for s in m.sides if bc.side.get(s) == OPEN]
        self.wall_sides = [s for s in m.sides if bc.side.get(s) == WALL]
        for s in m.sides:
            if bc.side.get(s) not in (WALL, OPEN):
                raise ValueError("side %d needs WALL or OPEN" % s)
        self.Bo = m.side_mass(self.open_sides)
        self.Bs = m.side_mass(self.wall_sides)
        # Dirichlet node sets
        self.dir = {}
        vset = set()
        for s in bc.pot_sides:
            vset |= set(m.side_nodes(s).tolist())
        if bc.electrodes:
            bn = m.side_nodes(BOTTOM)
            xs = m.X.ravel()[bn]
            for (x0, x1) in bc.electrodes:
                sel = bn[(xs >= x0 - 1e-12) & (xs <= x1 + 1e-12)]
                vset |= set(sel.tolist())
        self.dir["V"] = np.array(sorted(vset), dtype=np.int64)
        pset, uset = set(), set()
        for s in self.open_sides:
            pset |= set(m.side_nodes(s).tolist())
        for s in self.wall_sides:
            uset |= set(m.side_nodes(s).tolist())
        self.dir["P"] = np.array(sorted(pset), dtype=np.int64)
        self.dir["u"] = np.array(sorted(uset), dtype=np.int64)
        self.dir["psi"] = np.zeros(0, dtype=np.int64)
        self.dir["phi"] = np.zeros(0, dtype=np.int64)
        self.shift = {"V": 0.0, "psi": self.c["c_psi"], "phi": self.c["c_phi"],
                      "P": 0.0, "u": self.c["c_u"]}
        self._lu = {}
        self.lu_order = lu_order
        self.n = 0
        self.state = None

    # -- transforms along z (identity in 2D) -----------------------------------
    def fwd(self, f):
        """f_hat_k = (1/Nz) sum_j f_j exp(-i beta_k z_j), k = 0..Nz/2 (Sec. 3.2.2)."""
        if not self.is3d:
            return f
        return np.fft.rfft(f, axis=0) / self.Nz

    def inv(self, fh):
        if not self.is3d:
            return np.real(fh)
        return np.fft.irfft(fh * self.Nz, n=self.Nz, axis=0)

    def dz(self, f):
        """d/dz of a physical field by i beta_k (zero in 2D)."""
        if not self.is3d:
            return np.zeros_like(f)
        return self.inv(1j * self.beta_d[:, None] * self.fwd(f))

    def dz_hat(self, fh):
        if not self.is3d:
            return np.zeros_like(np.real(fh))
        return self.inv(1j * self.beta_d[:, None] * fh)

    # -- linear solves ------------------------------------------------------------
    def _factor(self, fam, k):
        key = (fam, k)
        if key in self._lu:
            return self._lu[key]
        m = self.m
        c = self.shift[fam] + self.beta[k] ** 2
        A = (m.Kst + c * m.M).tocsr()
        D = self.dir[fam]
        free = np.setdiff1d(np.arange(m.Ng), D)
        singular = (len(D) == 0) and c == 0.0
        if singular:
            mm = m.Mdiag.reshape(-1, 1)
            Ab = sp.bmat([[A, sp.csr_matrix(mm)], [sp.csr_matrix(mm.T), None]]).tocsc()
            lu = spla.splu(Ab, permc_spec=self.lu_order)
        else:
            lu = spla.splu(A[free][:, free].tocsc(), permc_spec=self.lu_order)
        ent = dict(A=A, free=free, D=D, lu=lu, singular=singular)
        self._lu[key] = ent
        return ent

    def solve(self, fam, k, b, gD=None):
        """Solve (K + c M) x = b for mode k with x = gD on the family's Dirichlet set.

        b and gD may be complex (3D); real and imaginary parts are solved alike.
        """
        if np.iscomplexobj(b) or (gD is not None and np.iscomplexobj(gD)):
            gr = None if gD is None else np.real(gD)
            gi = None if gD is None else np.imag(gD)
            return self.solve(fam, k, np.real(b), gr) + 1j * self.solve(fam, k, np.imag(b), gi)
        ent = self._factor(fam, k)
        m = self.m
        if ent["singular"]:
            bb = b - (b.sum() / m.Mdiag.sum()) * m.Mdiag   # project onto the range
            sol = ent["lu"].solve(np.concatenate([bb, [0.0]]))
            return sol[:-1]
        x = np.zeros(m.Ng)
        D, free = ent["D"], ent["free"]
        if len(D):
            x[D] = gD[D] if gD is not None else 0.0
            rhs = b[free] - ent["A"][free][:, D] @ x[D]
        else:
            rhs = b[free]
        x[free] = ent["lu"].solve(rhs)
        return x

    def solve_all(self, fam, bh, gDh=None):
        """Solve every mode (3D) or the single plane (2D)."""
        out = np.zeros_like(bh)
        for k in range(bh.shape[0]):
            out[k] = self.solve(fam, k, bh[k], None if gDh is None else gDh[k])
        return out

    # -- state --------------------------------------------------------------------
    def zeros(self):
        return np.zeros((self.Nz, self.m.Ng))

    def set_state(self, phi, u=None, P=None, V=None, prev=None, n0=0):
        """phi, V, P: (Nz, Ng) or (Ng,); u: tuple of 2 (2D) or 3 (3D) arrays.
        prev: optional dict with the same keys at level n-1 (else copies, reading R-bdf)."""
        def a(f):
            return self.zeros() if f is None else np.array(f, dtype=np.float64).reshape(self.Nz, self.m.Ng)
        ncomp = 3 if self.is3d else 2
        uu = [a(None) for _ in range(3)]
        if u is not None:
            for i in range(ncomp):
                uu[i] = a(u[i])
        cur = dict(phi=a(phi), P=a(P), V=a(V), u=uu)
        if prev is None:
            old = dict(phi=cur["phi"].copy(), P=cur["P"].copy(), V=cur["V"].copy(),
                       u=[x.copy() for x in cur["u"]])
        else:
            pu = [a(None) for _ in range(3)]
            for i in range(ncomp):
                pu[i] = a(prev["u"][i])
            old = dict(phi=a(prev["phi"]), P=a(prev.get("P")), V=a(prev["V"]), u=pu)
        self.state = dict(cur=cur, old=old)
        self.n = n0
        self.out = dict(psi=self.zeros(), E=[self.zeros() for _ in range(3)])

    def _src(self, src, name):
        if src is None or name not in src or src[name] is None:
            return self.zeros()
        return np.array(src[name], dtype=np.float64).reshape(self.Nz, self.m.Ng)

    # -- init potential (Remark 3.1) ---------------------------------------------
    def init_potential(self, src=None):
        """V^0 as the fixed point of Remark 3.1 (reading R-V0), 2D and 3D.

        2D: solve int eps(phi0) grad V . grad e = -int f_V e with V = Vd on the
        Dirichlet set.  3D: the variable coefficient couples modes, so the fixed
        point is iterated to convergence instead.
        """
        m, P = self.m, self.par
        phi0 = self.state["cur"]["phi"]
        fV = self._src(src, "fV")
        Vd = self._src(src, "Vd")
        if not self.is3d:
            el = P.eps(m.loc(phi0[0]))
            A = (m.Gx.T @ sp.diags(m.wq * el) @ m.Gx + m.Gy.T @ sp.diags(m.wq * el) @ m.Gy).tocsr()
            D = self.dir["V"]
            free = np.setdiff1d(np.arange(m.Ng), D)
            x = np.zeros(m.Ng)
            x[D] = Vd[0][D]
            b = -m.Mdiag * fV[0]
            x[free] = spla.spsolve(A[free][:, free].tocsc(), b[free] - A[free][:, D] @ x[D])
            V = x[None, :]
        else:
            V = self.iterate_potential(fV, Vd, tol=1e-13, maxit=20000)[0]
        self.state["cur"]["V"] = V.copy()
        self.state["old"]["V"] = V.copy()
        return V

    def iterate_potential(self, fV, Vd, tol, maxit):
        """The literal fixed-point iteration of Remark 3.1; returns (V, iterations)."""
        m, P = self.m, self.par
        eps0 = self.c["eps0"]
        phi0 = self.state["cur"]["phi"]
        V = self.zeros()
        for it in range(1, maxit + 1):
            Vn = self._potential_solve(phi0, V, fV, Vd)
            d = np.max(np.abs(Vn - V))
            V = Vn
            if d <= tol * max(1.0, np.max(np.abs(V))):
                return V, it
        return V, maxit

    def _potential_solve(self, phis, Vs, fV, Vd):
        """eq. (54)/(74): eps0 int grad V.grad e = -int (eps(phi*)-eps0) grad V* . grad e - int f_V e."""
        m, P = self.m, self.par
        eps0 = self.c["eps0"]
        A = np.zeros((self.Nz, m.Ng))
        B = np.zeros((self.Nz, m.Ng))
        dzV = self.dz(Vs)
        for j in range(self.Nz):
            r = P.eps(m.loc(phis[j])) - eps0
            A[j] = -m.weak_div(r * m.dx(Vs[j]), r * m.dy(Vs[j])) - m.Mdiag * fV[j]
            B[j] = m.Mdiag * (P.eps(phis[j]) - eps0) * dzV[j]
        bh = self.fwd(A) + 1j * self.beta_d[:, None] * self.fwd(B) if self.is3d else A
        Vh = self.solve_all("V", bh / eps0, self.fwd(Vd))
        return self.inv(Vh)

    # -- one time step ------------------------------------------------------------
    def step(self, src=None, equilibrium=False):
        """Advance (u, P, phi, V) from n to n+1 (Algorithm 1 / Algorithm 2).

        equilibrium=True runs the simpler system of Sec. 2.4 (eqs. 15c-d, 16):
        only the V, E, psi and phi sub-steps, with u = 0.
        """
        m, P, c = self.m, self.par, self.c
        cur, old = self.state["cur"], self.state["old"]
        if P.bdf == 2:
            star = lambda a, b: 2.0 * a - b
            hat = lambda a, b: 2.0 * a - 0.5 * b
        else:
            star = lambda a, b: a.copy()
            hat = lambda a, b: a.copy()
        g0, dt, lam, g1c = c["gamma0"], P.dt, P.lam, P.gamma1
        phis, phih = star(cur["phi"], old["phi"]), hat(cur["phi"], old["phi"])
        Vs = star(cur["V"], old["V"])
        us = [star(cur["u"][i], old["u"][i]) for i in range(3)]
        uh = [hat(cur["u"][i], old["u"][i]) for i in range(3)]
        Ps = star(cur["P"], old["P"])
        S = lambda n: self._src(src, n)
        Nz = self.Nz

        # ---- V^{n+1}: eq. (54) / (74) ----
        V = self._potential_solve(phis, Vs, S("fV"), S("Vd"))
        Vh = self.fwd(V)

        # ---- E^{n+1}: eq. (55) / (78), diagonal-mass projection ----
        Ex, Ey = self.zeros(), self.zeros()
        for j in range(Nz):
            Ex[j] = m.mass_local(m.dx(V[j])) / m.Mdiag
            Ey[j] = m.mass_local(m.dy(V[j])) / m.Mdiag
        Ez = self.dz_hat(Vh)                        # reading R-Ez
        E2 = Ex ** 2 + Ey ** 2 + Ez ** 2

        # ---- psi^{n+1}: eq. (56) / (75) ----
        cps, cph = c["c_psi"], c["c_phi"]
        g, g1, g2, g3 = S("g"), S("g1"), S("g2"), S("g3")
        dzphs = self.dz(phis)
        Q2 = P.h(phis) - c["S"] / P.eta ** 2 * phis - P.deps(phis) * E2 / (2.0 * lam)
        U = -g3 - P.theta_p_over_lam(phis)
        A = self.zeros()
        B = self.zeros()
        for j in range(Nz):
            adv = (m.loc(us[0][j]) * m.dx(phis[j]) + m.loc(us[1][j]) * m.dy(phis[j])
                   + m.loc(us[2][j] * dzphs[j]))
            Q1 = (m.loc(g[j]) - adv + m.loc(phih[j]) / dt) / (lam * g1c)
            A[j] = (-m.mass_local(Q1) + m.Kst @ Q2[j]
                    + self.Bo * (g1[j] + cps * g2[j]) + self.Bs * (g1[j] + cps * U[j]))
            B[j] = m.Mdiag * Q2[j]
        bh = self.fwd(A) + (self.beta[:, None] ** 2) * self.fwd(B)
        psih = self.solve_all("psi", bh)
        psi = self.inv(psih)

        # ---- phi^{n+1}: eq. (57) / (76), reading R-psi ----
        Bnd = self.zeros()
        for j in range(Nz):
            Bnd[j] = self.Bo * g2[j] + self.Bs * U[j]
        bh = -m.Mdiag[None, :] * psih + self.fwd(Bnd)
        phih1 = self.solve_all("phi", bh)
        phi = self.inv(phih1)

        if equilibrium:
            zero = [self.zeros() for _ in range(3)]
            self._rotate(phi=phi, V=V, P=self.zeros(), u=zero)
            self.out = dict(psi=psi, E=[Ex, Ey, Ez], phih=phih1, Vh=Vh)
            return self.fields()

        # ---- explicit momentum terms, eq. (49) and the G, Y, K, J, L of Sec. 3.2.2 ----
        rho0, num = c["rho0"], c["nu_m"]
        alpha = c["alpha"]
        Phi = psi - cps * phi - Q2                  # reading R-J
        dzphi = self.dz_hat(phih1)
        dzPhi = self.dz(Phi)
        dzPs = self.dz(Ps)
        dzus = [self.dz(us[i]) for i in range(3)]
        fx, fy, fz = S("fx"), S("fy"), S("fz")
        wx, wy, wz = S("wx"), S("wy"), S("wz")
        f1 = [S("f1x"), S("f1y"), S("f1z")]
        AP, BP = self.zeros(), self.zeros()
        keep = []
        for j in range(Nz):
            L = m.loc
            ph = L(phi[j])
            gph = [m.dx(phi[j]), m.dy(phi[j]), L(dzphi[j])]
            pc = np.clip(ph, -1.0, 1.0)             # reading R-clamp
            rho, mu = P.rho(pc), P.mu(pc)
            grho = [0.5 * (P.rho1 - P.rho2) * x for x in gph]
            gmu = [0.5 * (P.mu1 - P.mu2) * x for x in gph]
            gnu = [(rho * gmu[i] - mu * grho[i]) / rho ** 2 for i in range(3)]
            Jt = [0.5 * (P.rho1 - P.rho2) * lam * g1c * x
                  for x in (m.dx(Phi[j]), m.dy(Phi[j]), L(dzPhi[j]))]
            u = [L(us[i][j]) for i in range(3)]
            # grad u*: gu[i][k] = d_i u_k
            gu = [[m.dx(us[k][j]) for k in range(3)],
                  [m.dy(us[k][j]) for k in range(3)],
                  [L(dzus[k][j]) for k in range(3)]]
            om = [gu[1][2] - gu[2][1], gu[2][0] - gu[0][2], gu[0][1] - gu[1][0]]
            Dm = [[gu[i][k] + gu[k][i] for k in range(3)] for i in range(3)]
            gmD = [sum(gmu[i] * Dm[i][k] for i in range(3)) for k in range(3)]
            Nu = [sum(u[i] * gu[i][k] for i in range(3)) for k in range(3)]
            JgU = [sum(Jt[i] * gu[i][k] for i in range(3)) for k in range(3)]
            lap = L(psi[j]) - alpha * ph            # lap phi = psi - alpha phi (eq. 44b)
            e2 = L(E2[j])
            dep = P.deps(ph)
            gP = [m.dx(Ps[j]), m.dy(Ps[j]), L(dzPs[j])]
            ff = [L(fx[j]), L(fy[j]), L(fz[j])]
            uhl = [L(uh[i][j]) for i in range(3)]
            T = [(ff[i] - lam * lap * gph[i] - 0.5 * dep * e2 * gph[i] + gmD[i] - JgU[i]) / rho
                 + uhl[i] / dt - Nu[i] + (1.0 / rho0 - 1.0 / rho) * gP[i] for i in range(3)]
            cr = [gnu[1] * om[2] - gnu[2] * om[1],
                  gnu[2] * om[0] - gnu[0] * om[2],
                  gnu[0] * om[1] - gnu[1] * om[0]]
            G = [T[i] + cr[i] for i in range(3)]
            mr = mu / rho
            # pressure right side, eq. (58a) / (77a), reading R-Pbnd
            a = rho0 * m.weak_div(G[0], G[1]) - rho0 * m.side_tangential(m.sides, mr * om[2])
            b = -rho0 * m.mass_local(G[2])
            for s in m.sides:
                nxs, nys = NORMALS[s]
                b += rho0 * m.side_local([s], mr * (nxs * om[1] - nys * om[0]))
            for s in self.wall_sides:
                nxs, nys = NORMALS[s]
                a -= rho0 * g0 / dt * m.side_mass([s]) * (nxs * wx[j] + nys * wy[j])
            AP[j], BP[j] = a, b
            keep.append((G, om, mr))
        bh = self.fwd(AP) + 1j * self.beta_d[:, None] * self.fwd(BP) if self.is3d else AP
        self.rhs_P = bh
        Ph = self.solve_all("P", bh, self.fwd(S("f2")))
        Pn = self.inv(Ph)

        # ---- u^{n+1}: eq. (59) / (78) ----
        dzP = self.dz_hat(Ph)
        Au = [self.zeros() for _ in range(3)]
        Bu = [self.zeros() for _ in range(3)]
        for j in range(Nz):
            G, om, mr = keep[j]
            L = m.loc
            gPn = [m.dx(Pn[j]), m.dy(Pn[j]), L(dzP[j])]
            Y = [G[i] - gPn[i] / rho0 for i in range(3)]
            Kv = [(mr - num) * om[i] for i in range(3)]
            ax = m.mass_local(Y[0]) + m.weak_div(np.zeros_like(Kv[2]), Kv[2])
            ay = m.mass_local(Y[1]) - m.weak_div(Kv[2], np.zeros_like(Kv[2]))
            az = m.mass_local(Y[2]) - m.weak_div(-Kv[1], Kv[0])
            Au[0][j], Au[1][j], Au[2][j] = ax / num, ay / num, az / num
            Bu[0][j] = m.mass_local(Kv[1]) / num
            Bu[1][j] = -m.mass_local(Kv[0]) / num
            for s in self.open_sides:
                nxs, nys = NORMALS[s]
                Lv = [(mr - num) * nys * om[2], -(mr - num) * nxs * om[2],
                      (mr - num) * (nxs * om[1] - nys * om[0])]
                for i in range(3):
                    Au[i][j] += m.side_mass([s]) * f1[i][j] - m.side_local([s], Lv[i]) / num
        wd = [wx, wy, wz]
        un = []
        for i in range(3 if self.is3d else 2):
            bh = self.fwd(Au[i]) + 1j * self.beta_d[:, None] * self.fwd(Bu[i]) if self.is3d else Au[i]
            un.append(self.inv(self.solve_all("u", bh, self.fwd(wd[i]))))
        if not self.is3d:
            un.append(self.zeros())
        self._rotate(phi=phi, V=V, P=Pn, u=un)
        self.out = dict(psi=psi, E=[Ex, Ey, Ez], Ph=Ph, phih=phih1, Vh=Vh)
        return self.fields()

    def _rotate(self, **new):
        self.state["old"] = self.state["cur"]
        self.state["cur"] = dict(phi=new["phi"], V=new["V"], P=new["P"], u=new["u"])
        self.n += 1

    def fields(self):
        cur = self.state["cur"]
        d = dict(phi=cur["phi"], V=cur["V"], P=cur["P"], ux=cur["u"][0], uy=cur["u"][1],
                 uz=cur["u"][2], psi=self.out["psi"], Ex=self.out["E"][0],
                 Ey=self.out["E"][1], Ez=self.out["E"][2])
        return d

    # -- diagnostics ------------------------------------------------------------------
    def energy_terms(self, phi, u, E):
        """Discrete total energy of eq. (14), term by term, on the GLL quadrature:
        kinetic  int 1/2 rho(phi) |u|^2,
        mixing   int F(phi, grad phi) of eq. (double_well): 1/2 lambda phi^T K phi (assembled
                 stiffness, per plane) + 1/2 lambda int (d_z phi)^2 (3D) + lambda/(4 eta^2) int (phi^2-1)^2,
        electric int 1/2 D.E = 1/2 eps(phi) |E|^2 (D = eps E),
        wall     int over the wall sides of Theta(phi), eq. (theta_def), with gamma = sigma =
                 2 sqrt(2) lambda / (3 eta) and the constant (gamma_s1 + gamma_s2)/2 left out.
        phi: (planes, Ng); u, E: tuples of d (planes, Ng) arrays.  3D integrates over z with Lz/Nz."""
        m, P = self.m, self.par
        phi = np.atleast_2d(phi)
        wz = self.Lz / self.Nz if self.is3d else 1.0
        Md = m.Mdiag[None, :]
        rho = P.rho(phi)
        kin = 0.5 * np.sum(Md * rho * sum(np.atleast_2d(c) ** 2 for c in u)) * wz
        grad = sum(float(pl @ (m.Kst @ pl)) for pl in phi)
        if self.is3d:
            grad += float(np.sum(Md * self.dz(phi) ** 2))
        bulk = np.sum(Md * (phi * phi - 1.0) ** 2)
        mix = (0.5 * P.lam * grad + P.lam / (4.0 * P.eta ** 2) * bulk) * wz
        elec = 0.5 * np.sum(Md * P.eps(phi) * sum(np.atleast_2d(c) ** 2 for c in E)) * wz
        sigma = 2.0 * math.sqrt(2.0) * P.lam / (3.0 * P.eta)
        cth = math.cos(math.radians(P.theta_s_deg))
        theta = sigma * cth * phi * (phi * phi - 3.0) / 4.0
        wall = float(np.sum(self.Bs[None, :] * theta)) * wz if len(self.wall_sides) else 0.0
        return dict(kinetic=float(kin), mixing=float(mix), electric=float(elec), wall=wall,
                    total=float(kin + mix + elec + wall))

    def energy(self):
        """energy_terms of the current state (E from the last potential update)."""
        cur = self.state["cur"]
        return self.energy_terms(cur["phi"], cur["u"], self.out["E"])

    def march_to_equilibrium(self, src, tol, max_steps):
        """Equilibrium system (u = 0): step until r_m = max |phi^{m+1} - phi^m| <= tol
        (checked every step) or max_steps.  Returns (steps, r_m history)."""
        hist = []
        for n in range(max_steps):
            prev = self.state["cur"]["phi"].copy()
            self.step(src, equilibrium=True)
            r = float(np.max(np.abs(self.state["cur"]["phi"] - prev)))
            hist.append(r)
            if r <= tol:
                return n + 1, hist
        return max_steps, hist

    def mass(self, f=None):
        """int_h phi over the domain (per plane summed; 3D includes Lz/Nz)."""
        f = self.state["cur"]["phi"] if f is None else f
        s = float(np.sum(f * self.m.Mdiag[None, :]))
        return s * (self.Lz / self.Nz if self.is3d else 1.0)
