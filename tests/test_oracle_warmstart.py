"""Pins of the warm-start network's FP64 reference: closed forms of the convolution,
adjoint identities, finite differences, rounding, and the optimiser's first step."""
import math

import numpy as np
import pytest

from oracle import warmstart as ws


def test_gelu_values():
    """gelu(x) = x Phi(x): 0 at 0, Phi(1) at 1, -x Phi(-x) symmetry; gelu'(0) = 1/2 and
    gelu'(x) by central differences."""
    assert ws.gelu(0.0) == 0.0
    assert abs(ws.gelu(1.0) - 0.8413447460685429) < 1e-15
    x = np.linspace(-4, 4, 33)
    assert np.allclose(ws.gelu(x) - ws.gelu(-x), x, atol=1e-15)
    assert abs(ws.dgelu(0.0) - 0.5) < 1e-15
    h = 1e-6
    assert np.allclose(ws.dgelu(x), (ws.gelu(x + h) - ws.gelu(x - h)) / (2 * h), atol=1e-9)


def test_bf16_rounding():
    """Round to nearest bfloat16 (8 significant bits), ties to even; exact values stay."""
    one = 1.0
    ulp = 2.0 ** -7
    assert ws.bf16_round(np.array([one]))[0] == one
    assert ws.bf16_round(np.array([one + ulp / 2]))[0] == one            # tie -> even
    assert ws.bf16_round(np.array([one + 3 * ulp / 2]))[0] == one + 2 * ulp  # tie -> even
    assert ws.bf16_round(np.array([one + 0.6 * ulp]))[0] == one + ulp
    assert ws.bf16_round(np.array([-3.0]))[0] == -3.0
    r = np.random.default_rng(0).standard_normal(1000)
    q = ws.bf16_round(r)
    assert np.all(np.abs(q - r) <= 2.0 ** -8 * np.abs(r))    # unit roundoff of 8 significant bits


def _grid():
    # output 11 x 13 x 16: latent 2 x 2 x 2, last stage 16 x 16 x 16; z and y crop and pad
    # with zeros, x wraps (16 = 8 * 2, periodic)
    return ws.Grid(11, 13, 16, periodic=(True, False, True))


def _rand(rng, grid, scale=1.0):
    sh = ws.shapes(grid)
    sc = dict(W1=0.7, b1=0.1, W2=0.15, b2=0.1, W3=0.1, b3=0.1, K1=0.08, c1=0.1, K2=0.08, c2=0.1,
              K3=0.08, c3=0.1, wo=0.3, bo=0.2)
    return {k: rng.standard_normal(sh[k]) * sc[k] * scale for k in ws.NAMES}


def test_grid_shapes_and_wrap():
    g = _grid()
    assert g.lat == (2, 2, 2) and g.shape(3) == (16, 16, 16) and g.L0 == 16 * 8
    assert g.wrap == (False, False, True)       # z periodic but 11 != 16: zero padding
    assert ws.Grid(64, 73, 72, periodic=(True, False, True)).wrap == (True, False, True)


def test_conv_of_a_point_source():
    """A unit value at one point p0 in channel ci: conv(u)[p0 - d, co] = K[tap(d), co, ci] for
    every offset d, wrapped around the periodic axis and cut at the others; zero elsewhere."""
    rng = np.random.default_rng(3)
    K = rng.standard_normal((27, 16, 16))
    wrap = (False, False, True)
    for p0 in [(2, 3, 4), (0, 0, 0), (4, 4, 5)]:
        u = np.zeros((1, 5, 5, 6, 16))
        u[(0,) + p0 + (7,)] = 1.0
        out = ws.conv(u, K, wrap)
        expect = np.zeros_like(out)
        for dz in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    z, y, x = p0[0] - dz, p0[1] - dy, (p0[2] - dx) % 6
                    if 0 <= z < 5 and 0 <= y < 5:
                        expect[0, z, y, x, :] = K[9 * (dz + 1) + 3 * (dy + 1) + dx + 1, :, 7]
        assert np.array_equal(out, expect), p0


def test_adjoint_pairs():
    """<conv(u; K), g> = <u, conv_adjoint(g; K)> = sum K * conv_weight_grad(g, u), and
    <up(x), y> = <x, down(y)>, with and without wrapping axes."""
    rng = np.random.default_rng(4)
    for wrap in [(False, False, False), (True, False, True), (True, True, True)]:
        u = rng.standard_normal((2, 4, 6, 4, 16))
        g = rng.standard_normal((2, 4, 6, 4, 16))
        K = rng.standard_normal((27, 16, 16))
        lhs = np.sum(ws.conv(u, K, wrap) * g)
        assert abs(lhs - np.sum(u * ws.conv_adjoint(g, K, wrap))) < 1e-10 * abs(lhs)
        assert abs(lhs - np.sum(K * ws.conv_weight_grad(g, u, wrap))) < 1e-10 * abs(lhs)
    x = rng.standard_normal((2, 3, 2, 4, 16))
    y = rng.standard_normal((2, 6, 4, 8, 16))
    assert abs(np.sum(ws.up(x) * y) - np.sum(x * ws.down(y))) < 1e-12 * np.abs(y).sum()
    assert np.array_equal(ws.up(x)[:, 5, 3, 7], x[:, 2, 1, 3])


def test_loss_closed_form_with_zero_decoder():
    """Convolutions and biases zero: every x_s = gelu(0) = 0, so y = bo for every input,
    L = mean((bo - t)^2), dL/dbo = 2 sum_b (bo - t_b) / (B N), and W1..W3, K1, K2 get no
    gradient (dL/dx_s is zero below the last stage)."""
    rng = np.random.default_rng(1)
    grid = _grid()
    w = _rand(rng, grid)
    for s in (1, 2, 3):
        w["K%d" % s][:] = 0.0
        w["c%d" % s][:] = 0.0
    P = rng.uniform(-1, 1, (4, 3))
    T = rng.standard_normal((4, grid.N))
    c = ws.forward(w, P, grid)
    loss, g = ws.loss_and_grads(w, c, T, grid)
    assert np.array_equal(c["y"], np.broadcast_to(w["bo"], c["y"].shape))
    assert abs(loss - np.mean((w["bo"][None, :] - T) ** 2)) < 1e-14
    assert np.allclose(g["bo"], 2.0 * (4 * w["bo"] - T.sum(axis=0)) / (4 * grid.N), atol=1e-15)
    for k in ("W1", "W2", "W3", "K1", "K2"):
        assert not np.any(g[k]), k


def test_gradients_match_finite_differences():
    """Sampled entries of every weight group against central differences of the loss (FP64)."""
    rng = np.random.default_rng(2)
    grid = _grid()
    w = _rand(rng, grid)
    P = rng.uniform(-1, 1, (3, 3))
    T = rng.standard_normal((3, grid.N))
    loss, g = ws.loss_and_grads(w, ws.forward(w, P, grid), T, grid)
    h = 1e-5
    for k in ws.NAMES:
        flat = w[k].ravel()
        picks = rng.choice(flat.size, min(6, flat.size), replace=False)
        for i in picks:
            wp = {kk: vv.copy() for kk, vv in w.items()}
            wm = {kk: vv.copy() for kk, vv in w.items()}
            wp[k].ravel()[i] += h
            wm[k].ravel()[i] -= h
            lp = ws.loss_and_grads(wp, ws.forward(wp, P, grid), T, grid)[0]
            lm = ws.loss_and_grads(wm, ws.forward(wm, P, grid), T, grid)[0]
            fd = (lp - lm) / (2 * h)
            gi = g[k].ravel()[i]
            assert abs(fd - gi) < 1e-6 * max(abs(fd), 1e-3 * np.abs(g[k]).max()), (k, i, fd, gi)


def test_blob_round_trip():
    rng = np.random.default_rng(5)
    grid = _grid()
    w = _rand(rng, grid)
    b = ws.to_blob(w)
    assert b.size == sum(int(np.prod(s)) for s in ws.shapes(grid).values())
    w2 = ws.from_blob(b, grid)
    assert all(np.array_equal(w[k], w2[k]) for k in ws.NAMES)


def test_adam_first_step_moves_by_lr():
    """At t = 1 the bias-corrected moments are g and g^2, so each weight moves by
    -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    w = _rand(rng, _grid())
    g = {k: rng.standard_normal(v.shape) for k, v in w.items()}
    w0 = {k: v.copy() for k, v in w.items()}
    ws.adam(w, g, {}, 1e-3, 1)
    for k in w:
        assert np.allclose(w[k] - w0[k], -1e-3 * g[k] / (np.abs(g[k]) + 1e-8), atol=1e-15)


def test_mass_projection_and_scaling():
    rng = np.random.default_rng(4)
    y = rng.standard_normal(50)
    wts = rng.uniform(0.1, 1, 50)
    z = ws.mass_project(y, wts, 3.5)
    assert abs(np.sum(wts * z) - 3.5) < 1e-12
    assert np.allclose(np.diff(z - y), 0.0, atol=1e-15)
    assert np.allclose(ws.scale_params(0.0, 1.5, 60.0), [-1, -1, -1])
    assert np.allclose(ws.scale_params(2.0, 40.0, 120.0), [1, 1, 1])
    assert abs(ws.scale_params(1.0, math.sqrt(60.0), 90.0)).max() < 1e-12
