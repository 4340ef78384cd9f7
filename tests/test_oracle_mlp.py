"""Pins for the oracle's variance-surrogate MLP (oracle/mlp.py).

* the parameter count of the 4 -> 256 -> 256 -> 256 -> 1 network;
* forward: zero weights give the output bias; a one-unit path gives the closed form
  w4 silu(w3 silu(w2 silu(w1 x + b1)))...;
* gradient: central finite differences of the loss, for every parameter group;
* Adam: the first step moves every parameter by -lr sign(g) (bias-corrected moments), and a
  1-D quadratic is minimised;
* initialisation: uniform within +-1/sqrt(fan_in), from the Philox stream.
"""
import numpy as np
import pytest

from oracle import mlp


def test_parameter_count():
    assert mlp.NPARAM == 4 * 256 + 256 + 2 * (256 * 256 + 256) + 256 + 1 == 133121


def test_init_is_bounded_and_deterministic():
    a = mlp.init_params(3)
    b = mlp.init_params(3)
    c = mlp.init_params(4)
    assert np.array_equal(a, b) and not np.array_equal(a, c)
    p = mlp.unpack(a)
    assert np.abs(p["W1"]).max() <= 0.5 and np.abs(p["W1"]).max() > 0.45
    assert np.abs(p["W2"]).max() <= 1 / 16 and np.abs(p["W2"]).max() > 0.06
    assert abs(p["W2"].mean()) < 1e-3 and abs(p["W2"].std() - (1 / 16) / np.sqrt(3)) < 1e-3


def test_forward_special_cases():
    th = np.zeros(mlp.NPARAM)
    p = mlp.unpack(th)
    p["b4"][0] = 0.7
    x = np.random.default_rng(0).normal(size=(5, 4))
    assert np.allclose(mlp.forward(th, x), 0.7)
    # one path through unit 0 of every layer
    th = np.zeros(mlp.NPARAM)
    p = mlp.unpack(th)
    p["W1"][0] = [0.5, -1.0, 0.25, 2.0]
    p["b1"][0] = 0.1
    p["W2"][0, 0] = 1.5
    p["W3"][0, 0] = -0.75
    p["b3"][0] = 0.2
    p["w4"][0, 0] = 3.0
    s = lambda z: z / (1 + np.exp(-z))
    h1 = s(x @ np.array([0.5, -1.0, 0.25, 2.0]) + 0.1)
    h2 = s(1.5 * h1)
    h3 = s(-0.75 * h2 + 0.2)
    # the other units see silu(0) = 0
    assert np.allclose(mlp.forward(th, x), 3.0 * h3, rtol=1e-14, atol=1e-15)


def test_gradient_matches_finite_differences():
    rng = np.random.default_rng(1)
    th = mlp.init_params(7)
    x = rng.normal(size=(9, 4))
    t = rng.normal(size=9)
    L, g = mlp.loss_and_grad(th, x, t)
    offs = np.cumsum([0] + [int(np.prod(s)) for _, s in mlp.SHAPES])
    h = 1e-6
    for gi in range(len(mlp.SHAPES)):
        idx = rng.integers(offs[gi], offs[gi + 1], size=min(6, offs[gi + 1] - offs[gi]))
        for j in idx:
            e = np.zeros_like(th)
            e[j] = h
            fd = (mlp.loss_and_grad(th + e, x, t)[0] - mlp.loss_and_grad(th - e, x, t)[0]) / (2 * h)
            assert abs(fd - g[j]) <= 1e-6 * max(1.0, abs(g[j])) + 1e-9, (mlp.SHAPES[gi][0], j, fd, g[j])


def test_adam_first_step_and_quadratic():
    opt = mlp.Adam(3, lr=0.01)
    th = np.array([1.0, -2.0, 0.5])
    g = np.array([0.3, -4.0, 1e-3])
    th1 = opt.step(th, g)
    assert np.allclose(th1 - th, -0.01 * np.sign(g), rtol=1e-4)
    # minimise (x - 3)^2 from 0
    opt = mlp.Adam(1, lr=0.05)
    x = np.array([0.0])
    for _ in range(2000):
        x = opt.step(x, 2 * (x - 3.0))
    assert abs(x[0] - 3.0) < 1e-3


def test_training_fits_a_smooth_function():
    rng = np.random.default_rng(2)
    x = rng.uniform(-1, 1, size=(64, 4))
    t = np.sin(x[:, 0]) + x[:, 1] * x[:, 2] - 0.5 * x[:, 3]
    th, losses = mlp.train(mlp.init_params(1), x, t, 300, lr=3e-3)
    assert losses[-1] < 0.02 * losses[0]


def test_features():
    edges = np.array([1.0, 4.0, 9.0, 16.0])
    X = mlp.features(edges, np.array([[2, 1, 0]]), 0.9)
    assert np.allclose(X, [[np.log(12.0), np.log(6.0), np.log(2.0), 0.9]])
