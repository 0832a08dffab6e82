"""Pins of the FP64 selector-network oracle: central differences, GELU and BCE closed forms, Adam."""
import math

import numpy as np
import pytest
from scipy.special import erf

from oracle import mlp


def test_gelu_matches_erf_definition_and_derivative():
    x = np.linspace(-6, 6, 101)
    assert np.allclose(mlp.gelu(x), [0.5 * v * (1 + math.erf(v / math.sqrt(2))) for v in x], rtol=1e-14, atol=1e-15)
    h = 1e-6
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.allclose(mlp.gelu_grad(x), fd, rtol=1e-7, atol=1e-9)


def test_bce_closed_form():
    z = np.array([-30.0, -2.0, 0.0, 1.5, 40.0])
    y = np.array([1.0, 0.0, 1.0, 1.0, 0.0])
    pw = 3.0
    sig = 1 / (1 + np.exp(-z))
    direct = -(pw * y * np.log(np.maximum(sig, 1e-300)) + (1 - y) * np.log(np.maximum(1 - sig, 1e-300)))
    # the extreme rows saturate the naive formula; compare on the finite ones and check the stable ones
    assert mlp.bce_with_logits(z[1:4], y[1:4], pw) == pytest.approx(direct[1:4].mean(), rel=1e-13)
    assert mlp.bce_with_logits(np.array([-30.0]), np.array([1.0]), pw) == pytest.approx(pw * 30.0, rel=1e-12)
    assert mlp.bce_with_logits(np.array([40.0]), np.array([0.0]), pw) == pytest.approx(40.0, rel=1e-12)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(0)
    p = mlp.init_params(1) * 0.7
    X = rng.normal(size=(37, 8))
    y = (rng.uniform(size=37) < 0.3).astype(float)
    _, g = mlp.loss_and_grad(p, X, y, 2.5)
    idx = rng.choice(mlp.NPARAM, size=120, replace=False)
    idx = np.concatenate([idx, [0, 511, 512, 575, 576, 4671, 4672, 4735, 4736, 4799, 4800]])
    h = 1e-6
    for k in idx:
        e = np.zeros(mlp.NPARAM)
        e[k] = h
        fd = (mlp.loss_and_grad(p + e, X, y, 2.5)[0] - mlp.loss_and_grad(p - e, X, y, 2.5)[0]) / (2 * h)
        assert g[k] == pytest.approx(fd, rel=1e-5, abs=1e-9), k


def test_layout_and_adam():
    p = np.arange(mlp.NPARAM, dtype=float)
    W1, b1, W2, b2, W3, b3 = mlp.unpack(p)
    assert W1[0, 1] == 1 and b1[0] == 512 and W2[0, 0] == 576 and b2[0] == 4672 and W3[0] == 4736 and b3 == 4800
    assert np.array_equal(mlp.pack(W1, b1, W2, b2, W3, b3), p)
    # first Adam step moves every parameter by lr against the gradient sign (bias-corrected)
    g = np.linspace(-1, 1, mlp.NPARAM) + 1e-3
    q, m1, m2 = mlp.adam_step(np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), np.zeros(mlp.NPARAM), g, 1e-2, 0.9, 0.999,
                              1e-12, 1)
    assert np.allclose(q, -1e-2 * np.sign(g), rtol=1e-6)


def test_budgeted_labels():
    c = np.array([0.5, 1e-4, 2e-4, 0.3, 3e-4, 0.2])
    lab = mlp.budgeted_keep_labels(c, 5e-4)
    # 1e-4 + 2e-4 = 3e-4 <= 5e-4; adding 3e-4 exceeds the budget
    assert lab.tolist() == [1, 0, 0, 1, 1, 1]
    assert mlp.budgeted_keep_labels(c, 0.0).tolist() == [1] * 6
