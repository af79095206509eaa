"""Pins of the FP64 surrogate network reference (oracle/mlp.py) against
facts that do not come from the code itself: finite differences of the loss,
the normal CDF's table value and symmetry, Adam's closed-form steps, and a
degenerate network."""
import math

import numpy as np

import lbm_inputs as L
from oracle import mlp


def test_gelu_values_and_symmetry():
    assert mlp.gelu(np.array([0.0]))[0] == 0.0
    # GELU(1) = Phi(1), the standard normal CDF at one standard deviation
    assert abs(mlp.gelu(np.array([1.0]))[0] - 0.8413447460685429) < 1e-15
    x = np.linspace(-6, 6, 97)
    # Phi(-x) = 1 - Phi(x)  =>  GELU(-x) = GELU(x) - x
    assert np.allclose(mlp.gelu(-x), mlp.gelu(x) - x, rtol=0, atol=1e-14)
    assert mlp.gelu(np.array([40.0]))[0] == 40.0 and mlp.gelu(np.array([-40.0]))[0] == 0.0
    h = 1e-5
    fd = (mlp.gelu(x + h) - mlp.gelu(x - h)) / (2 * h)
    assert np.abs(fd - mlp.gelu_grad(x)).max() < 1e-9


def _small():
    dims = [7, 16, 16, 16, 16, 12]
    shapes = mlp.layer_shapes(7, 16, 4, 12)
    assert [s[1] for s in shapes] + [12] == dims
    theta = L.mlp_init(dims, seed=4)
    rng = np.random.default_rng(5)
    xn = rng.uniform(-1, 1, (5, 7))
    tn = rng.normal(size=(5, 12))
    return shapes, theta, xn, tn


def test_gradient_matches_finite_differences_small_net():
    shapes, theta, xn, tn = _small()
    _, g = mlp.loss_and_grad(theta, shapes, xn, tn)
    h = 1e-6
    fd = np.empty_like(theta)
    for k in range(theta.size):
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd[k] = (mlp.loss(tp, shapes, xn, tn) - mlp.loss(tm, shapes, xn, tn)) / (2 * h)
    assert np.linalg.norm(g - fd) / np.linalg.norm(fd) < 1e-7
    assert np.abs(g - fd).max() < 1e-8


def test_gradient_matches_finite_differences_full_size_sampled():
    shapes = mlp.layer_shapes()
    dims = [7, 512, 512, 512, 512, 512]
    theta = L.mlp_init(dims, seed=6)
    assert theta.size == mlp.n_params(shapes) == 1054720
    rng = np.random.default_rng(7)
    xn = rng.uniform(-1, 1, (3, 7))
    tn = rng.normal(size=(3, 512))
    _, g = mlp.loss_and_grad(theta, shapes, xn, tn)
    # sample entries of every layer's weights and biases
    offs, k = [], 0
    for o, i in shapes:
        offs += list(k + rng.integers(0, o * i, 4)) + list(k + o * i + rng.integers(0, o, 2))
        k += o * i + o
    h = 1e-5
    for k in offs:
        tp, tm = theta.copy(), theta.copy()
        tp[k] += h
        tm[k] -= h
        fd = (mlp.loss(tp, shapes, xn, tn) - mlp.loss(tm, shapes, xn, tn)) / (2 * h)
        # FD rounding is ~eps L / h ~ 2e-11; a wrong term is off by O(|fd|)
        assert abs(g[k] - fd) <= 2e-10 + 1e-6 * abs(fd), (k, g[k], fd)


def test_adam_closed_forms():
    rng = np.random.default_rng(8)
    theta = rng.normal(size=50)
    g = rng.normal(size=50)
    opt = mlp.Adam(50, lr=1e-2)
    t1 = opt.step(theta, g)
    # first step: m_hat = g, v_hat = g^2, so the step is lr g / (|g| + eps)
    assert np.abs(t1 - (theta - 1e-2 * g / (np.abs(g) + 1e-8))).max() < 1e-15
    # a constant gradient keeps m_hat = g and v_hat = g^2 at every step
    t = t1
    for _ in range(9):
        t = opt.step(t, g)
    assert np.abs(t - (theta - 10 * 1e-2 * g / (np.abs(g) + 1e-8))).max() < 1e-13


def test_zero_hidden_weights_give_the_last_bias():
    shapes, theta, xn, _ = _small()
    layers = mlp.unpack(theta, shapes)
    for W, _ in layers[1:]:
        W[:] = 0.0
    y, _, _ = mlp.forward(theta, shapes, xn)
    assert np.array_equal(y, np.broadcast_to(layers[-1][1], y.shape))


def test_input_normalisation_maps_box_corners():
    lo, hi = L.SURROGATE_LO, L.SURROGATE_HI
    assert np.array_equal(mlp.normalise_inputs(lo, lo, hi), -np.ones(7))
    assert np.allclose(mlp.normalise_inputs(hi, lo, hi), np.ones(7), atol=1e-15)
    assert math.isclose(float(mlp.normalise_inputs((lo + hi) / 2, lo, hi)[2]), 0.0, abs_tol=1e-15)
