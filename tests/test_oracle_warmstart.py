"""Pins of the warm-start network's FP64 reference: closed forms, finite differences,
rounding, and the optimiser's first step."""
import math

import numpy as np
import pytest

from oracle import warmstart as ws


def _weights(rng, n_out=7, h1=5, h2=6):
    return dict(W1=rng.standard_normal((h1, 3)) * 0.7, b1=rng.standard_normal(h1) * 0.1,
                W2=rng.standard_normal((h2, h1)) * 0.5, b2=rng.standard_normal(h2) * 0.1,
                W3=rng.standard_normal((n_out, h2)) * 0.4, b3=rng.standard_normal(n_out) * 0.2)


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


def test_loss_closed_form_with_zero_decoder():
    """W3 = 0: y = b3 for every input, so L = mean((b3 - t)^2) and dL/db3 = 2 mean_b(b3 - t)/N."""
    rng = np.random.default_rng(1)
    w = _weights(rng)
    w["W3"][:] = 0.0
    P = rng.uniform(-1, 1, (4, 3))
    T = rng.standard_normal((4, 7))
    c = ws.forward(w, P)
    loss, g = ws.loss_and_grads(w, c, T)
    assert abs(loss - np.mean((w["b3"][None, :] - T) ** 2)) < 1e-14
    assert np.allclose(g["b3"], 2.0 * (w["b3"] - T.mean(axis=0)) / 7, atol=1e-15)
    assert np.allclose(g["W1"], 0.0) and np.allclose(g["W2"], 0.0)


def test_gradients_match_finite_differences():
    """Every gradient entry against central differences of the loss (FP64)."""
    rng = np.random.default_rng(2)
    w = _weights(rng)
    P = rng.uniform(-1, 1, (3, 3))
    T = rng.standard_normal((3, 7))
    loss, g = ws.loss_and_grads(w, ws.forward(w, P), T)
    h = 1e-6
    for k in w:
        for idx in np.ndindex(w[k].shape):
            wp = {kk: vv.copy() for kk, vv in w.items()}
            wm = {kk: vv.copy() for kk, vv in w.items()}
            wp[k][idx] += h
            wm[k][idx] -= h
            lp, _ = ws.loss_and_grads(wp, ws.forward(wp, P), T)
            lm, _ = ws.loss_and_grads(wm, ws.forward(wm, P), T)
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[k][idx]) < 1e-7 * max(1.0, abs(fd)), (k, idx, fd, g[k][idx])


def test_adam_first_step_moves_by_lr():
    """At t = 1 the bias-corrected moments are g and g^2, so each weight moves by
    -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    w = _weights(rng)
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
