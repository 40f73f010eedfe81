"""Float64 reference of the surrogate network of the learned energy grid (test infrastructure only).

The network maps (E, disorder sigma, Nx, Ny) to (log DOS, log T): fully connected layers
widths[0] -> ... -> widths[-1], tanh on every hidden layer, identity on the output.
Parameters are one flat vector: per layer the weight matrix W (rows = outputs, row-major)
followed by the bias b.  The loss is the mean squared error over all outputs of all samples.
The optimiser is Adam (Kingma and Ba, 2015): bias-corrected first and second moment estimates.

Written directly from those definitions in numpy float64: forward pass, reverse-mode
derivative of the loss by the chain rule, Adam update.  Shares no code with the HIP path.
"""
from __future__ import annotations

import numpy as np


def unpack(params, widths):
    """[(W, b)] views of the flat parameter vector."""
    p = np.asarray(params, dtype=np.float64)
    out, o = [], 0
    for a, b in zip(widths[:-1], widths[1:]):
        W = p[o:o + a * b].reshape(b, a)
        o += a * b
        out.append((W, p[o:o + b]))
        o += b
    if o != p.size:
        raise ValueError("parameter count does not match the widths")
    return out


def n_params(widths):
    return sum(a * b + b for a, b in zip(widths[:-1], widths[1:]))


def forward(params, widths, x, keep=False):
    """Network output y [n, widths[-1]] (and the list of layer inputs when keep=True)."""
    h = np.asarray(x, dtype=np.float64)
    layers = unpack(params, widths)
    hs = [h]
    for k, (W, b) in enumerate(layers):
        z = h @ W.T + b
        h = np.tanh(z) if k + 1 < len(layers) else z
        hs.append(h)
    return (h, hs) if keep else h


def loss(params, widths, x, t):
    y = forward(params, widths, x)
    d = y - np.asarray(t, dtype=np.float64)
    return float(np.mean(d * d))


def grads(params, widths, x, t):
    """Flat gradient of the loss with respect to the parameters (chain rule, layer by layer)."""
    y, hs = forward(params, widths, x, keep=True)
    t = np.asarray(t, dtype=np.float64)
    layers = unpack(params, widths)
    delta = 2.0 * (y - t) / y.size          # d loss / d y
    g = []
    for k in range(len(layers) - 1, -1, -1):
        W, _ = layers[k]
        h_in = hs[k]
        g.append((delta.T @ h_in, delta.sum(axis=0)))
        if k > 0:
            delta = (delta @ W) * (1.0 - h_in * h_in)   # through tanh: h_in = tanh(z)
    flat = []
    for dW, db in reversed(g):
        flat.append(dW.ravel())
        flat.append(db)
    return np.concatenate(flat)


def adam_step(p, g, m, v, step, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update; step counts from 1.  Returns (p, m, v)."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    return p - lr * mhat / (np.sqrt(vhat) + eps), m, v


def train(params, widths, x, t, steps, lr=1e-3, batch=None, order=None, beta1=0.9, beta2=0.999, eps=1e-8):
    """Adam on the loss; step s uses rows order[s*batch:(s+1)*batch] (all rows if order is None)."""
    p = np.asarray(params, dtype=np.float64).copy()
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    x = np.asarray(x, dtype=np.float64)
    t = np.asarray(t, dtype=np.float64)
    hist = []
    for s in range(steps):
        if order is None:
            xs, ts = x, t
        else:
            idx = np.asarray(order[s * batch:(s + 1) * batch])
            xs, ts = x[idx], t[idx]
        hist.append(loss(p, widths, xs, ts))
        p, m, v = adam_step(p, grads(p, widths, xs, ts), m, v, s + 1, lr, beta1, beta2, eps)
    return p, np.array(hist)
