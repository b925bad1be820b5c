"""FP64 reference of the learned warm start's network (test infrastructure: only tests and
the benchmark's CPU baseline use it; the library never does).

The network maps the three parameters of an equilibrium problem (voltage, permittivity
ratio, contact angle; scaled to [-1, 1]) to the equilibrium phase field on a grid of
nz x ny x nx values (C order, z slowest).  It is a small convolutional decoder:

    a1 = W1 p + b1,   h1 = gelu(a1)                     64 units
    a2 = W2 h1 + b2,  h2 = gelu(a2)                     128 units
    x0 = W3 h2 + b3                                     latent grid Z0 x Y0 x X0, 16 channels
    for s = 1, 2, 3:
        u_s = up(x_{s-1})                               nearest-neighbour doubling of each axis
        a_s = conv(u_s; K_s) + c_s,  x_s = gelu(a_s)    3x3x3 convolution, 16 -> 16 channels
    y  = crop(sum_c wo[c] x_3[..., c]) + bo             the corner nz x ny x nx of the last grid

with Z0 = ceil(nz / 8) (likewise Y0, X0), gelu(x) = x Phi(x) (Phi the standard normal
distribution function) and the loss L = mean over the batch and the outputs of (y - t)^2.
Grids are channel-last: x_s[b, z, y, x, c].  The convolution is

    conv(u; K)[p, co] = sum over d in {-1, 0, 1}^3 and ci of K[tap(d), co, ci] u[p + d, ci],
    tap(d) = 9 (dz + 1) + 3 (dy + 1) + (dx + 1),

where a neighbour p + d outside the grid wraps around along an axis that wraps (the
axis is periodic and 8 Z0 = nz exactly) and counts as zero along any other axis.
Training uses Adam.

The library rounds to bfloat16 the operands of its matrix-core products: h2 and W3 (latent
layer), the latent x0 and every activation x_s (the next layer's input), the convolution
weights, and the gradients dL/da_s and dL/dx0 that enter the backward products; bf16=True
mirrors exactly those roundings (round to nearest, ties to even) so that the two can be
compared closely.  The weight blob is the concatenation, in this order, of
W1 (64 x 3), b1, W2 (128 x 64), b2, W3 (L0 x 128, L0 = 16 Z0 Y0 X0), b3 (L0),
K1 (27 x 16 x 16), c1, K2, c2, K3, c3, wo (16), bo (nz ny nx).
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)
H1, H2, CH, STAGES = 64, 128, 16, 3
NAMES = ("W1", "b1", "W2", "b2", "W3", "b3", "K1", "c1", "K2", "c2", "K3", "c3", "wo", "bo")


def gelu(x):
    return 0.5 * x * (1.0 + erf(x / SQRT2))


def dgelu(x):
    return 0.5 * (1.0 + erf(x / SQRT2)) + x * np.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def bf16_round(a):
    """Round float32 values to the nearest bfloat16 (ties to even), returned as float64."""
    a32 = np.ascontiguousarray(a, dtype=np.float32)
    u = a32.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    return r.astype(np.uint32).view(np.float32).astype(np.float64)


def scale_params(V, eps_ratio, theta_deg, vmax=2.0, rmin=1.5, rmax=40.0, tmin=60.0, tmax=120.0):
    """The network inputs: each parameter mapped linearly (the ratio logarithmically) to
    [-1, 1] over its sampling range."""
    return np.array([2.0 * V / vmax - 1.0,
                     2.0 * (math.log(eps_ratio) - math.log(rmin)) / (math.log(rmax) - math.log(rmin)) - 1.0,
                     2.0 * (theta_deg - tmin) / (tmax - tmin) - 1.0])


class Grid:
    """Output grid (nz, ny, nx) with per-axis periodicity; latent and stage shapes."""

    def __init__(self, nz, ny, nx, periodic=(False, False, False)):
        self.out = (nz, ny, nx)
        self.lat = tuple(-(-n // 8) for n in self.out)
        self.wrap = tuple(bool(p) and 8 * l == n for p, l, n in zip(periodic, self.lat, self.out))
        self.L0 = CH * int(np.prod(self.lat))
        self.N = nz * ny * nx

    def shape(self, s):
        return tuple(l << s for l in self.lat)


def shapes(grid):
    """Weight shapes in blob order."""
    return dict(W1=(H1, 3), b1=(H1,), W2=(H2, H1), b2=(H2,), W3=(grid.L0, H2), b3=(grid.L0,),
                K1=(27, CH, CH), c1=(CH,), K2=(27, CH, CH), c2=(CH,), K3=(27, CH, CH), c3=(CH,),
                wo=(CH,), bo=(grid.N,))


def to_blob(w):
    return np.concatenate([np.ravel(w[k]) for k in NAMES])


def from_blob(b, grid):
    out, o = {}, 0
    for k, sh in shapes(grid).items():
        n = int(np.prod(sh))
        out[k] = np.asarray(b[o:o + n], dtype=np.float64).reshape(sh)
        o += n
    return out


def _offsets():
    return [(t // 9 - 1, (t // 3) % 3 - 1, t % 3 - 1) for t in range(27)]


def _shift(u, d, wrap):
    """v[p] = u[p + d] over the spatial axes (1..3) of u (batch, z, y, x, c); a neighbour
    outside the grid wraps along a wrapping axis and is zero along any other."""
    v = u
    for ax, (dd, w) in enumerate(zip(d, wrap), start=1):
        if dd == 0:
            continue
        v = np.roll(v, -dd, axis=ax)
        if not w:
            idx = [slice(None)] * v.ndim
            idx[ax] = slice(-1, None) if dd > 0 else slice(0, 1)
            v[tuple(idx)] = 0.0
    return v


def conv(u, K, wrap):
    """conv(u; K)[p, co] = sum_d sum_ci K[tap(d), co, ci] u[p + d, ci]."""
    out = np.zeros(u.shape[:-1] + (K.shape[1],))
    for t, d in enumerate(_offsets()):
        out += _shift(u, d, wrap) @ K[t].T
    return out


def conv_adjoint(g, K, wrap):
    """The adjoint of u -> conv(u; K): r[q, ci] = sum_d sum_co K[tap(d), co, ci] g[q - d, co]."""
    out = np.zeros(g.shape[:-1] + (K.shape[2],))
    for t, d in enumerate(_offsets()):
        out += _shift(g, tuple(-x for x in d), wrap) @ K[t]
    return out


def conv_weight_grad(g, u, wrap):
    """dL/dK[tap(d), co, ci] = sum over batch and p of g[p, co] u[p + d, ci]."""
    G = g.reshape(-1, g.shape[-1])
    return np.stack([G.T @ _shift(u, d, wrap).reshape(-1, u.shape[-1]) for d in _offsets()])


def up(x):
    """Nearest-neighbour doubling of the three spatial axes."""
    return x.repeat(2, axis=1).repeat(2, axis=2).repeat(2, axis=3)


def down(g):
    """The adjoint of up: each coarse value collects the sum of its eight children."""
    b, z, y, x, c = g.shape
    return g.reshape(b, z // 2, 2, y // 2, 2, x // 2, 2, c).sum(axis=(2, 4, 6))


def forward(w, P, grid, bf16=False):
    """w: weight dict; P: (B, 3).  Returns the cache with y (B, N)."""
    q = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    P = np.asarray(P, dtype=np.float64)
    B = P.shape[0]
    a1 = P @ w["W1"].T + w["b1"]
    h1 = gelu(a1)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = gelu(a2)
    h2q, W3q = q(h2), q(w["W3"])
    x0 = h2q @ W3q.T + w["b3"]
    xs = [q(x0.reshape((B,) + grid.lat + (CH,)))]     # layer inputs as the products see them
    Kq = [q(w["K%d" % s]) for s in (1, 2, 3)]
    a = []
    for s in range(STAGES):
        pre = conv(up(xs[-1]), Kq[s], grid.wrap) + w["c%d" % (s + 1)]
        a.append(pre)
        xs.append(q(gelu(pre)))
    nz, ny, nx = grid.out
    y = (xs[-1][:, :nz, :ny, :nx, :] @ w["wo"]).reshape(B, -1) + w["bo"]
    return dict(P=P, a1=a1, h1=h1, a2=a2, h2=h2, h2q=h2q, W3q=W3q, xs=xs, Kq=Kq, a=a, y=y)


def loss_and_grads(w, cache, T, grid, bf16=False):
    """Loss and its gradients with respect to every weight (backpropagation)."""
    q = bf16_round if bf16 else (lambda a: np.asarray(a, dtype=np.float64))
    T = np.asarray(T, dtype=np.float64)
    y = cache["y"]
    B, N = y.shape
    d = y - T
    loss = float(np.mean(d * d))
    dy = 2.0 * d / (B * N)
    g = {"bo": dy.sum(axis=0)}
    nz, ny, nx = grid.out
    x3 = cache["xs"][-1]
    dyg = dy.reshape(B, nz, ny, nx)
    g["wo"] = np.einsum("bzyx,bzyxc->c", dyg, x3[:, :nz, :ny, :nx, :])
    dx = np.zeros(x3.shape)
    dx[:, :nz, :ny, :nx, :] = dyg[..., None] * w["wo"]
    for s in range(STAGES - 1, -1, -1):
        da = q(dx * dgelu(cache["a"][s]))
        u = up(cache["xs"][s])
        g["K%d" % (s + 1)] = conv_weight_grad(da, u, grid.wrap)
        g["c%d" % (s + 1)] = da.sum(axis=(0, 1, 2, 3))
        dx = down(conv_adjoint(da, cache["Kq"][s], grid.wrap))
    dx0 = dx.reshape(B, -1)
    g["b3"] = dx0.sum(axis=0)
    dq = q(dx0)
    g["W3"] = dq.T @ cache["h2q"]
    dh2 = dq @ cache["W3q"]
    da2 = dh2 * dgelu(cache["a2"])
    g["W2"] = da2.T @ cache["h1"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ w["W2"]
    da1 = dh1 * dgelu(cache["a1"])
    g["W1"] = da1.T @ cache["P"]
    g["b1"] = da1.sum(axis=0)
    return loss, g


def adam(w, g, state, lr, t, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (t counts from 1) on every weight, in place; state holds m and v."""
    for k in w:
        m = state.setdefault("m_" + k, np.zeros_like(w[k]))
        v = state.setdefault("v_" + k, np.zeros_like(w[k]))
        m[...] = beta1 * m + (1.0 - beta1) * g[k]
        v[...] = beta2 * v + (1.0 - beta2) * g[k] * g[k]
        mh = m / (1.0 - beta1 ** t)
        vh = v / (1.0 - beta2 ** t)
        w[k] = w[k] - lr * mh / (np.sqrt(vh) + eps)
    return w


def mass_project(y, weights, mass):
    """Shift y by a constant so that sum(weights * y) = mass (the discrete integral)."""
    return y + (mass - float(np.sum(weights * y))) / float(np.sum(weights))
