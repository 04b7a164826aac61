"""Pins of the NumPy classifier oracle: central finite differences for the
hand-derived backward pass, the closed form of a first Adam step, the GELU
(tanh form) against the exact erf form, and the loss at a known logit."""
import math

import numpy as np
from scipy.special import erf

from oracle import mlp


def _batch(seed, B=32):
    rng = np.random.default_rng(seed)
    X = rng.normal(size=(B, mlp.NIN)) * 2.0 + 0.5
    y = (rng.uniform(size=B) < 0.4).astype(float)
    w = rng.uniform(0.5, 2.0, size=B)
    mean = rng.normal(size=mlp.NIN) * 0.3
    std = rng.uniform(0.5, 2.0, size=mlp.NIN)
    return X, y, w, mean, std


def test_parameter_count():
    assert mlp.NPARAM == 16 * 64 + 64 + 64 * 64 + 64 + 64 + 1 == 5313


def test_backward_matches_central_differences():
    X, y, w, mean, std = _batch(1)
    th = mlp.init_params(7) + np.random.default_rng(8).normal(size=mlp.NPARAM) * 0.05
    loss, g = mlp.loss_and_grad(th, X, y, w, mean, std)
    rng = np.random.default_rng(9)
    idx = rng.choice(mlp.NPARAM, size=200, replace=False)
    idx = np.concatenate([idx, [mlp.NPARAM - 1, 0, 16 * 64 + 3]])
    eps = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = eps
        lp, _ = mlp.loss_and_grad(th + e, X, y, w, mean, std)
        lm, _ = mlp.loss_and_grad(th - e, X, y, w, mean, std)
        fd = (lp - lm) / (2 * eps)
        assert abs(fd - g[k]) <= 1e-7 + 1e-5 * abs(fd), (k, fd, g[k])


def test_first_adam_step_closed_form():
    """After one step from zero moments, m_hat = g and v_hat = g^2, so each
    parameter moves by -lr g / (|g| + eps)."""
    rng = np.random.default_rng(3)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    new, m, v = mlp.adam_step(th, np.zeros(50), np.zeros(50), g, 1, lr=0.01)
    assert np.allclose(new, th - 0.01 * g / (np.abs(g) + 1e-8), rtol=0, atol=1e-15)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_gelu_tanh_form_close_to_erf_form():
    z = np.linspace(-6, 6, 2001)
    exact = 0.5 * z * (1.0 + erf(z / math.sqrt(2.0)))
    assert np.abs(mlp.gelu(z) - exact).max() < 1e-3
    assert mlp.gelu(0.0) == 0.0


def test_loss_at_known_logit():
    """All weights zero: every logit equals b3, so the loss is the weighted mean
    of softplus(-b3) (y = 1) and softplus(b3) (y = 0)."""
    th = np.zeros(mlp.NPARAM)
    th[-1] = 0.3
    X, y, w, mean, std = _batch(4, B=16)
    loss, _ = mlp.loss_and_grad(th, X, y, w, mean, std)
    sp = lambda s: math.log1p(math.exp(s))
    want = np.mean(w * np.where(y == 1, sp(-0.3), sp(0.3)))
    assert abs(loss - want) < 1e-15
    assert np.allclose(mlp.forward(th, X, mean, std), 0.3)
