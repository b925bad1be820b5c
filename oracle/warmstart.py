"""FP64 reference of the learned warm start's network (test infrastructure: only tests and
the benchmark's CPU baseline use it; the library never does).

The network maps the three parameters of an equilibrium problem (voltage, permittivity
ratio, contact angle; scaled to [-1, 1]) to the equilibrium phase field on the grid:

    a1 = W1 p + b1,   h1 = gelu(a1)            (H1 units)
    a2 = W2 h1 + b2,  h2 = gelu(a2)            (H2 units)
    y  = W3 h2 + b3                            (N outputs: the field)

with gelu(x) = x Phi(x) (Phi the standard normal distribution function) and the loss
L = mean over the batch and the outputs of (y - t)^2.  Training uses Adam.  The library
evaluates W3 h2 with BF16 operands (FP32 master weights, FP32 accumulation) and rounds dL/dy
to BF16 for its two large products; bf16=True mirrors those roundings (round to nearest,
ties to even) so that the two can be compared closely.
"""
import math

import numpy as np
from scipy.special import erf

SQRT2 = math.sqrt(2.0)


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


def forward(w, P, bf16=False):
    """w: dict W1, b1, W2, b2, W3, b3; P: (B, 3).  Returns the cache with y (B, N)."""
    P = np.asarray(P, dtype=np.float64)
    a1 = P @ w["W1"].T + w["b1"]
    h1 = gelu(a1)
    a2 = h1 @ w["W2"].T + w["b2"]
    h2 = gelu(a2)
    if bf16:
        h2q, W3q = bf16_round(h2), bf16_round(w["W3"])
    else:
        h2q, W3q = h2, w["W3"]
    y = h2q @ W3q.T + w["b3"]
    return dict(P=P, a1=a1, h1=h1, a2=a2, h2=h2, h2q=h2q, W3q=W3q, y=y)


def loss_and_grads(w, cache, T, bf16=False):
    """Loss and its gradients with respect to every weight (backpropagation)."""
    T = np.asarray(T, dtype=np.float64)
    y = cache["y"]
    B, N = y.shape
    d = y - T
    loss = float(np.mean(d * d))
    dy = 2.0 * d / (B * N)
    gb3 = dy.sum(axis=0)
    dyq = bf16_round(dy) if bf16 else dy
    gW3 = dyq.T @ cache["h2q"]
    dh2 = dyq @ cache["W3q"]
    da2 = dh2 * dgelu(cache["a2"])
    gW2 = da2.T @ cache["h1"]
    gb2 = da2.sum(axis=0)
    dh1 = da2 @ w["W2"]
    da1 = dh1 * dgelu(cache["a1"])
    gW1 = da1.T @ cache["P"]
    gb1 = da1.sum(axis=0)
    return loss, dict(W1=gW1, b1=gb1, W2=gW2, b2=gb2, W3=gW3, b3=gb3)


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
