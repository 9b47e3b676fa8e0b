"""Pins of the CPU oracle of the learned gate (oracle/mlp.py): back-propagation
against finite differences, the activation against the exact Gaussian error
linear unit, closed-form loss and Adam cases, and the harvest definition on
states whose chi is known."""
import math

import numpy as np
import pytest
from scipy.stats import norm

from oracle import mlp as M
from paper_2507_20461_amd import inputs


def test_parameter_count():
    assert M.NPARAM == 6849
    p = M.init(0)
    assert np.array_equal(M.pack(*M.unpack(p)), p)


def test_gradient_matches_central_differences():
    rng = np.random.default_rng(3)
    p = M.init(1) + 0.05 * rng.standard_normal(M.NPARAM)
    X = rng.standard_normal((7, 40))
    y = rng.uniform(0, 1, 7)
    g = M.grad(p, X, y)
    h = 1e-6
    fd = np.empty(M.NPARAM)
    for k in range(M.NPARAM):
        e = np.zeros(M.NPARAM)
        e[k] = h
        fd[k] = (M.loss(p + e, X, y) - M.loss(p - e, X, y)) / (2 * h)
    scale = np.abs(fd).max()
    assert np.abs(g - fd).max() < 1e-7 * max(scale, 1.0), np.abs(g - fd).max()


def test_gelu_is_the_tanh_form_of_x_phi():
    u = np.linspace(-6, 6, 2001)
    exact = u * norm.cdf(u)
    assert np.abs(M.gelu(u) - exact).max() < 1e-3          # the tanh form's own error (~2e-4)
    assert M.gelu(np.array([0.0]))[0] == 0.0
    assert abs(M.gelu(np.array([30.0]))[0] - 30.0) < 1e-12
    assert abs(M.gelu(np.array([-30.0]))[0]) < 1e-12
    h = 1e-6
    fd = (M.gelu(u + h) - M.gelu(u - h)) / (2 * h)
    assert np.abs(M.gelu_d(u) - fd).max() < 1e-8


def test_zero_network_loss_is_log2():
    p = np.zeros(M.NPARAM)
    X = np.random.default_rng(0).standard_normal((5, 40))
    for y in (np.zeros(5), np.ones(5), np.full(5, 0.3)):
        assert abs(M.loss(p, X, y) - math.log(2.0)) < 1e-15
    z, _ = M.forward(p, X)
    assert np.all(M.sigmoid(z) == 0.5)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -1e-3, 2e-2])
    p1, m, v = M.adam(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, 1e-3)
    assert np.allclose(p1, -1e-3 * np.sign(g), rtol=1e-4)


def test_harvest_of_a_constant_state():
    W = np.empty((4, 6, 7))
    W[:] = np.array([1.2, 0.3, -0.4, 2.5])[:, None, None]
    for d in (0, 1):
        X, _ = M.harvest(W, np.zeros((8, 6, 7)), d, 1, 1.0 / 7)
        assert np.all(X == 0.0)


def test_harvest_inputs_and_targets(oracle):
    # quadrants: cells next to a jump have tiny chi, cells far from any jump
    # chi = 1; value features lie in [-1, 1] with a zero centre
    n = 24
    W, dW, _ = inputs.quadrants_2d(n, n, 1)
    prm = oracle.params(ndim=2, bc=1)
    for d in (0, 1):
        _, chi = oracle.normal_faces(prm, W, dW, d)
        X, y = M.harvest(W, dW, d, 1, 1.0 / n, chi)
        Xv = X.reshape(n * n, 4, 10)
        assert np.abs(Xv[:, :, 0:5]).max() <= 1.0 and np.all(Xv[:, :, 2] == 0.0)
        y2 = y.reshape(n, n)
        idx = np.arange(n)
        near = (np.abs(idx - (n // 2 - 0.5)) < 1.0)    # the two cells on either side of the mid line
        far = (np.abs(idx - (n // 2 - 0.5)) > 3.0)
        line = near[None, :] if d == 0 else near[:, None]
        assert np.all(y2[np.broadcast_to(line, (n, n))] < 1e-6)
        assert np.all(y2[np.ix_(far, far)] == 1.0)
