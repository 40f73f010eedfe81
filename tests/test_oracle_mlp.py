"""Pins of the float64 network oracle (finite differences, closed forms, Adam's first step)."""
import numpy as np

import oracle
from oracle import mlp as om


def _rand(widths, seed):
    rng = np.random.default_rng(seed)
    return rng.normal(0, 0.5, om.n_params(widths))


def test_param_count_of_the_surrogate():
    assert om.n_params((4, 256, 256, 2)) == 4 * 256 + 256 + 256 * 256 + 256 + 256 * 2 + 2 == 67586


def test_gradient_matches_central_differences():
    widths = (4, 5, 6, 2)
    p = _rand(widths, 0)
    rng = np.random.default_rng(1)
    x, t = rng.normal(size=(7, 4)), rng.normal(size=(7, 2))
    g = om.grads(p, widths, x, t)
    h = 1e-6
    fd = np.empty_like(p)
    for i in range(p.size):
        e = np.zeros_like(p)
        e[i] = h
        fd[i] = (om.loss(p + e, widths, x, t) - om.loss(p - e, widths, x, t)) / (2 * h)
    assert np.abs(g - fd).max() <= 1e-7 * max(1.0, np.abs(fd).max())


def test_one_hidden_unit_closed_form():
    # y = w2 tanh(w1 x + b1) + b2, loss = (y - t)^2 for one sample
    w1, b1, w2, b2 = 0.7, -0.2, 1.3, 0.4
    x, t = 0.9, 0.1
    p = np.array([w1, b1, w2, b2])
    a = np.tanh(w1 * x + b1)
    y = w2 * a + b2
    assert abs(om.forward(p, (1, 1, 1), [[x]])[0, 0] - y) < 1e-15
    r = 2 * (y - t)
    want = np.array([r * w2 * (1 - a * a) * x, r * w2 * (1 - a * a), r * a, r])
    assert np.allclose(om.grads(p, (1, 1, 1), [[x]], [[t]]), want, rtol=1e-14, atol=0)


def test_adam_first_step_is_lr_times_sign():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p, m, v = om.adam_step(np.zeros(4), g, np.zeros(4), np.zeros(4), 1, lr=0.01, eps=1e-8)
    assert np.allclose(p, -0.01 * g / (np.abs(g) + 1e-8), rtol=1e-14, atol=0)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_adam_reaches_least_squares_on_a_linear_model():
    # no hidden layer: y = W x + b is linear, the loss is a convex quadratic with a closed-form minimum
    rng = np.random.default_rng(3)
    x = rng.normal(size=(40, 3))
    t = x @ np.array([[0.5], [-1.0], [2.0]]) + 0.3 + 0.01 * rng.normal(size=(40, 1))
    p, hist = om.train(np.zeros(4), (3, 1), x, t, steps=3000, lr=0.02)
    A = np.hstack([x, np.ones((40, 1))])
    sol = np.linalg.lstsq(A, t[:, 0], rcond=None)[0]
    assert np.abs(p - sol).max() < 1e-4
    assert hist[-1] < hist[0]


def test_minibatch_order_selects_rows():
    widths = (2, 3, 1)
    p0 = _rand(widths, 4)
    rng = np.random.default_rng(5)
    x, t = rng.normal(size=(6, 2)), rng.normal(size=(6, 1))
    order = np.array([5, 1, 3, 0])
    pa, ha = om.train(p0, widths, x, t, steps=2, batch=2, order=order)
    pb, hb = om.train(p0, widths, x[[5, 1]], t[[5, 1]], steps=1)
    assert abs(ha[0] - hb[0]) < 1e-15
