"""Surrogate network kernels (through the C ABI) against the float64 oracle."""
import numpy as np
import pytest
import torch

import oracle.mlp as om
import paper_1702_05167_amd as pkg
from paper_1702_05167_amd import learned_grid as lg

pytestmark = pytest.mark.gpu

W = (4, 256, 256, 2)


def _setup(seed, n):
    rng = np.random.default_rng(seed)
    p = lg.xavier_init(W, seed).astype(np.float64)
    p += np.where(p == 0, rng.normal(0, 0.1, p.size), 0.0)      # non-zero biases
    p = p.astype(np.float32)
    x = rng.uniform(-1, 1, (n, 4)).astype(np.float32)
    t = rng.normal(0, 1, (n, 2)).astype(np.float32)
    return p, x, t


def rel(a, b):
    return np.abs(np.asarray(a, np.float64) - b).max() / np.abs(b).max()


@pytest.mark.parametrize("n", [1, 63, 333, 2000])
def test_forward_matches_oracle(ctx, n):
    p, x, _ = _setup(0, n)
    net = pkg.MLP(ctx, W)
    net.set_params(p)
    y = net.forward(x).cpu().numpy()
    ref = om.forward(p.astype(np.float64), W, x.astype(np.float64))
    assert rel(y, ref) <= 2e-6, rel(y, ref)
    assert np.array_equal(net.get_params().cpu().numpy(), p)


@pytest.mark.parametrize("n", [1, 333, 2000])
def test_gradients_match_oracle(ctx, n):
    p, x, t = _setup(1, n)
    net = pkg.MLP(ctx, W)
    net.set_params(p)
    g, loss = net.grads(x, t)
    g = g.cpu().numpy()
    ref = om.grads(p.astype(np.float64), W, x.astype(np.float64), t.astype(np.float64))
    lref = om.loss(p.astype(np.float64), W, x.astype(np.float64), t.astype(np.float64))
    assert abs(loss - lref) <= 1e-6 * lref
    for off, shp, boff, bn in net.layout():
        k = shp[0] * shp[1]
        assert rel(g[off:off + k], ref[off:off + k]) <= 1e-4, ("W", shp)
        assert rel(g[boff:boff + bn], ref[boff:boff + bn]) <= 1e-4, ("b", bn)


def test_adam_training_follows_oracle(ctx):
    p, x, t = _setup(2, 500)
    net = pkg.MLP(ctx, W)
    net.set_params(p)
    rng = np.random.default_rng(9)
    order = np.concatenate([rng.permutation(500)[:400] for _ in range(5)]).astype(np.int32)   # 20 steps of 100
    hist = net.train(x, t, steps=20, lr=1e-3, batch=100, order=order)
    p_ref, h_ref = om.train(p.astype(np.float64), W, x.astype(np.float64), t.astype(np.float64), steps=20,
                            lr=1e-3, batch=100, order=order)
    assert np.abs(hist - h_ref).max() <= 1e-4 * h_ref.max(), (hist, h_ref)
    q = net.get_params().cpu().numpy().astype(np.float64)
    step = q - p
    step_ref = p_ref - p
    # Adam moves every parameter by about lr per step; FP32 gradients may flip the direction
    # only where the gradient is at rounding level
    assert np.linalg.norm(step - step_ref) <= 2e-2 * np.linalg.norm(step_ref)


def test_full_batch_training_reduces_loss(ctx):
    rng = np.random.default_rng(4)
    x = rng.uniform(-1, 1, (1000, 4)).astype(np.float32)
    t = np.stack([np.sin(3 * x[:, 0]) * x[:, 1], np.cos(2 * x[:, 2]) + x[:, 3] ** 2], 1).astype(np.float32)
    net = pkg.MLP(ctx, W)
    net.set_params(lg.xavier_init(W, 4))
    hist = net.train(x, t, steps=300, lr=3e-3)
    assert hist[-1] < 0.05 * hist[0], (hist[0], hist[-1])


def test_bad_sample_index_gives_nan_loss(ctx):
    p, x, t = _setup(3, 50)
    net = pkg.MLP(ctx, W)
    net.set_params(p)
    order = np.full(10, 50, np.int32)          # one past the end: the gather writes NaN rows
    hist = net.train(x, t, steps=1, batch=10, order=order)
    assert np.isnan(hist[0])
