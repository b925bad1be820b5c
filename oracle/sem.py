"""C0 spectral-element building blocks for the oracle (Sec. 3.2.1, function space X_h).

Reading adopted where the paper is silent: Lagrange polynomials through the
K+1 Gauss-Lobatto-Legendre (GLL) points per direction, with the same points used
as quadrature (collocation), so the mass matrix is diagonal.

Everything is plain and assembled: element loops build SciPy sparse matrices.
Layouts:
  global nodal field  g = iy*Nx + ix          (Ny x Nx array, row-major)
  element-local value q = (e*(K+1) + b)*(K+1) + a,  e = ey*nx + ex,
                      a = local x index, b = local y index.
"""
import numpy as np
import scipy.sparse as sp


def legendre(K, x):
    """Return (P_K(x), P_K'(x)) by the three-term recurrence."""
    x = np.asarray(x, dtype=np.float64)
    p0 = np.ones_like(x)
    if K == 0:
        return p0, np.zeros_like(x)
    p1 = x.copy()
    for n in range(1, K):
        p0, p1 = p1, ((2 * n + 1) * x * p1 - n * p0) / (n + 1)
    # derivative from (1-x^2) P_K' = K (P_{K-1} - x P_K); valid off +-1
    with np.errstate(divide="ignore", invalid="ignore"):
        dp = K * (p0 - x * p1) / (1.0 - x * x)
    end = np.abs(np.abs(x) - 1.0) < 1e-300
    dp = np.where(end, np.sign(x) ** (K + 1) * K * (K + 1) / 2.0, dp)
    return p1, dp


def gll(K):
    """GLL nodes (ascending) and weights for polynomial order K >= 1.

    Interior nodes are the roots of P_K', found by Newton's method on
    f(x) = P_K'(x) using f'(x) = (2x P_K' - K(K+1) P_K)/(1-x^2).
    Weights: w_j = 2 / (K(K+1) P_K(x_j)^2).
    """
    if K < 1:
        raise ValueError("K must be >= 1")
    x = -np.cos(np.pi * np.arange(K + 1) / K)  # Chebyshev-Lobatto start
    xi = x[1:-1].copy()
    for _ in range(100):
        p, dp = legendre(K, xi)
        d2p = (2 * xi * dp - K * (K + 1) * p) / (1 - xi * xi)
        step = dp / d2p
        xi -= step
        if np.max(np.abs(step), initial=0.0) < 1e-16:
            break
    x[1:-1] = xi
    x[0], x[-1] = -1.0, 1.0
    p, _ = legendre(K, x)
    w = 2.0 / (K * (K + 1) * p * p)
    return x, w


def diff_matrix(K):
    """D[i, j] = l_j'(x_i) for the Lagrange basis through the GLL nodes.

    Closed form for GLL points: D_ij = P_K(x_i) / (P_K(x_j) (x_i - x_j)) for i != j,
    D_00 = -K(K+1)/4, D_KK = K(K+1)/4, other diagonal entries 0.
    """
    x, _ = gll(K)
    p, _ = legendre(K, x)
    D = np.zeros((K + 1, K + 1))
    for i in range(K + 1):
        for j in range(K + 1):
            if i != j:
                D[i, j] = p[i] / (p[j] * (x[i] - x[j]))
    D[0, 0] = -K * (K + 1) / 4.0
    D[K, K] = K * (K + 1) / 4.0
    return D


# side ids used throughout: 0 bottom (y=ymin), 1 top (y=ymax), 2 left, 3 right
BOTTOM, TOP, LEFT, RIGHT = 0, 1, 2, 3
NORMALS = {BOTTOM: (0.0, -1.0), TOP: (0.0, 1.0), LEFT: (-1.0, 0.0), RIGHT: (1.0, 0.0)}


class Mesh2D:
    """Tensor-product mesh of nx x ny axis-aligned rectangles, order K.

    xb (nx+1) and yb (ny+1) are the element breakpoints.  With periodic_x the
    nodes at x = xb[-1] are identified with those at x = xb[0].
    """

    def __init__(self, xb, yb, K, periodic_x=False):
        self.xb = np.asarray(xb, dtype=np.float64)
        self.yb = np.asarray(yb, dtype=np.float64)
        self.K = int(K)
        self.periodic_x = bool(periodic_x)
        self.nx, self.ny = len(self.xb) - 1, len(self.yb) - 1
        K = self.K
        self.Nx = self.nx * K + 1 - (1 if self.periodic_x else 0)
        self.Ny = self.ny * K + 1
        self.Ng = self.Nx * self.Ny
        self.ne = self.nx * self.ny
        self.nq = (K + 1) ** 2
        self.Nl = self.ne * self.nq
        self.xi, self.w = gll(K)
        self.D = diff_matrix(K)
        self.hx = np.diff(self.xb)
        self.hy = np.diff(self.yb)
        # 1D global coordinates
        x = np.zeros(self.nx * K + 1)
        for ex in range(self.nx):
            x[ex * K:(ex + 1) * K + 1] = self.xb[ex] + 0.5 * self.hx[ex] * (self.xi + 1.0)
        y = np.zeros(self.ny * K + 1)
        for ey in range(self.ny):
            y[ey * K:(ey + 1) * K + 1] = self.yb[ey] + 0.5 * self.hy[ey] * (self.xi + 1.0)
        self.x1 = x[: self.Nx].copy()
        self.y1 = y.copy()
        self.X, self.Y = np.meshgrid(self.x1, self.y1)  # (Ny, Nx)
        self._build()

    # -- indexing -------------------------------------------------------------
    def gix(self, ex, a):
        i = ex * self.K + a
        return i % self.Nx if self.periodic_x else i

    def giy(self, ey, b):
        return ey * self.K + b

    def _build(self):
        K, nq = self.K, self.nq
        rows_z, cols_z = [], []
        rx, cx, vx = [], [], []
        ry, cy, vy = [], [], []
        wq = np.zeros(self.Nl)
        self.loc2glob = np.zeros(self.Nl, dtype=np.int64)
        self.xq = np.zeros(self.Nl)
        self.yq = np.zeros(self.Nl)
        for ey in range(self.ny):
            for ex in range(self.nx):
                e = ey * self.nx + ex
                hx, hy = self.hx[ex], self.hy[ey]
                J = hx * hy / 4.0
                for b in range(K + 1):
                    for a in range(K + 1):
                        q = e * nq + b * (K + 1) + a
                        g = self.giy(ey, b) * self.Nx + self.gix(ex, a)
                        self.loc2glob[q] = g
                        rows_z.append(q)
                        cols_z.append(g)
                        wq[q] = J * self.w[a] * self.w[b]
                        self.xq[q] = self.xb[ex] + 0.5 * hx * (self.xi[a] + 1)
                        self.yq[q] = self.yb[ey] + 0.5 * hy * (self.xi[b] + 1)
                        for p in range(K + 1):
                            # d/dx at (a,b) uses nodes (p,b)
                            rx.append(q)
                            cx.append(self.giy(ey, b) * self.Nx + self.gix(ex, p))
                            vx.append(2.0 / hx * self.D[a, p])
                            # d/dy at (a,b) uses nodes (a,p)
                            ry.append(q)
                            cy.append(self.giy(ey, p) * self.Nx + self.gix(ex, a))
                            vy.append(2.0 / hy * self.D[b, p])
        shp = (self.Nl, self.Ng)
        self.Z = sp.csr_matrix((np.ones(len(rows_z)), (rows_z, cols_z)), shape=shp)
        self.Gx = sp.csr_matrix((vx, (rx, cx)), shape=shp)
        self.Gy = sp.csr_matrix((vy, (ry, cy)), shape=shp)
        self.wq = wq
        W = sp.diags(wq)
        self.W = W
        self.Mdiag = np.asarray(self.Z.T @ wq).ravel()
        self.M = sp.diags(self.Mdiag).tocsr()
        self.Kst = (self.Gx.T @ W @ self.Gx + self.Gy.T @ W @ self.Gy).tocsr()
        # boundary edges: element-local edge quadrature weights per side
        self.side_w = {}
        for s in (BOTTOM, TOP, LEFT, RIGHT):
            if self.periodic_x and s in (LEFT, RIGHT):
                continue
            sw = np.zeros(self.Nl)
            if s in (BOTTOM, TOP):
                ey = 0 if s == BOTTOM else self.ny - 1
                b = 0 if s == BOTTOM else K
                for ex in range(self.nx):
                    e = ey * self.nx + ex
                    for a in range(K + 1):
                        sw[e * nq + b * (K + 1) + a] = 0.5 * self.hx[ex] * self.w[a]
            else:
                ex = 0 if s == LEFT else self.nx - 1
                a = 0 if s == LEFT else K
                for ey in range(self.ny):
                    e = ey * self.nx + ex
                    for b in range(K + 1):
                        sw[e * nq + b * (K + 1) + a] = 0.5 * self.hy[ey] * self.w[b]
            self.side_w[s] = sw
        self.sides = sorted(self.side_w)

    # -- element-local helpers -------------------------------------------------
    def loc(self, f):
        """Global nodal field (Ny, Nx) -> element-local values (Nl,)."""
        return np.asarray(self.Z @ np.asarray(f).ravel())

    def dx(self, f):
        return np.asarray(self.Gx @ np.asarray(f).ravel())

    def dy(self, f):
        return np.asarray(self.Gy @ np.asarray(f).ravel())

    def mass_local(self, floc):
        """int_h f e_i for an element-local f: Z^T W f  -> (Ng,)."""
        return np.asarray(self.Z.T @ (self.wq * floc))

    def weak_div(self, fx_loc, fy_loc):
        """int_h F . grad e_i for element-local F: Gx^T W Fx + Gy^T W Fy."""
        return np.asarray(self.Gx.T @ (self.wq * fx_loc) + self.Gy.T @ (self.wq * fy_loc))

    def side_nodes(self, s):
        """Global indices of the nodes on side s."""
        sw = self.side_w[s]
        return np.unique(self.loc2glob[sw > 0])

    def side_mass(self, sides):
        """Diagonal boundary mass over the union of sides: int_{sides} f e_i (f nodal)."""
        d = np.zeros(self.Ng)
        for s in sides:
            d += np.asarray(self.Z.T @ self.side_w[s]).ravel()
        return d

    def side_local(self, sides, floc):
        """int_{sides} f e_i for an element-local f (values taken from the element
        owning each boundary edge)."""
        out = np.zeros(self.Ng)
        for s in sides:
            out += np.asarray(self.Z.T @ (self.side_w[s] * floc))
        return out

    def side_tangential(self, sides, floc):
        """int_{sides} f (n x omega_hat) . grad e_i  for a scalar (2D) omega factor
        folded into floc:  (n x (0,0,w)) = w (n_y, -n_x, 0), so the integrand is
        f * (n_y d/dx e_i - n_x d/dy e_i), with grad e_i taken in the owning element."""
        out = np.zeros(self.Ng)
        for s in sides:
            nxs, nys = NORMALS[s]
            v = self.side_w[s] * floc
            out += np.asarray(nys * (self.Gx.T @ v) - nxs * (self.Gy.T @ v))
        return out
