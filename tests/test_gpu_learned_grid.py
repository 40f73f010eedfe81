"""Learned energy grid end to end (small devices): surrogate trained on the solver's outputs by
the library's kernels, proposal judged by the HSC solve."""
import numpy as np
import pytest

import synth
import paper_1702_05167_amd as pkg
from paper_1702_05167_amd import learned_grid as lg

pytestmark = pytest.mark.gpu


def _item(N, sigma, seed):
    dev = synth.learned_grid_device(N, sigma, seed)
    return dict(tree=pkg.Tree.from_device(dev, leaf_side=4, transverse=True), n_sites=dev.n, sigma=sigma, nx=N, ny=N)


def test_totals_match_host_sums(ctx):
    dev = synth.learned_grid_device(8, 0.3, 5)
    tree = pkg.Tree.from_device(dev, leaf_side=4, transverse=True)
    out = pkg.solve(ctx, tree, np.array([-1.3, 0.05, 2.5]), want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL |
                    pkg.HSC_SPECTRAL_LR, precision=0)
    t = pkg.totals(ctx, out, dev.n).cpu().numpy()
    gr, gl, sp = (out[k].cpu().numpy() for k in ("gr", "gl", "spectral"))
    assert np.allclose(t[:, 0], -gr.imag.sum(1) / np.pi, rtol=1e-13, atol=0)
    assert np.allclose(t[:, 1], gl.imag.sum(1) / (2 * np.pi), rtol=1e-13, atol=1e-300)
    assert np.allclose(t[:, 2], sp.sum((1, 2)) / (2 * np.pi), rtol=1e-13, atol=1e-300)


def test_learned_grid_small_devices(ctx):
    rng = np.random.default_rng(0)
    train = []
    for d in range(8):
        N = int(rng.integers(8, 13))
        train.append(_item(N, float(rng.uniform(0, 0.5)), 2000 + d))
    X, Y = lg.dataset(ctx, train, 40, seed=1)
    sur = lg.Surrogate(ctx, seed=0)
    hist = sur.fit(X, Y, epochs=200, batch=80)
    print("loss", hist[0], "->", hist[-1])
    assert hist[-20:].mean() < 0.2 * hist[:20].mean()
    r = lg.study(ctx, sur, _item(12, 0.3, 100), np.linspace(-6, 6, 1024), 128, (-2.0, 2.0), budget=16,
                 sweep=(16, 32, 64))
    for k in ("dense", "guided_proposal", "guided", "uniform", "uniform_in_support"):
        print(k, r[k])
    print("sweep", r["sweep"])
    # the surrogate-chosen grid (plus solver-judged refinement) needs far fewer solves than the
    # dense grid and beats the plain uniform grid of the same size
    assert r["guided"]["solves"] < 0.5 * r["dense"]["solves"]
    assert r["guided"]["rel_err"] < r["uniform"]["rel_err"]
    assert r["guided"]["rel_err"] < 2e-3


def test_learned_grid_equal_cost(ctx):
    # what the trained network gains over the method without it, at equal numbers of in-band
    # solves: the surrogate-proposed grid plus solver-judged refinement (a quarter of the solves)
    # against the evenly spaced in-band grid of the same size.  The integrand of a disordered 12^3
    # cube is a comb of resonances the smooth surrogate cannot place, so at small budgets (<= 64
    # solves) either grid's error is a matter of where the resonances fall; the test asserts the
    # regime where a grid reliably reaches the charge tolerance (1e-4 at every larger budget of the
    # sweep): there the guided grid wins at every budget and gets there with fewer solves
    rng = np.random.default_rng(0)
    train = []
    for d in range(8):
        N = int(rng.integers(8, 13))
        train.append(_item(N, float(rng.uniform(0, 0.5)), 2000 + d))
    X, Y = lg.dataset(ctx, train, 40, seed=1)
    sur = lg.Surrogate(ctx, seed=0)
    sur.fit(X, Y, epochs=200, batch=80)
    r = lg.equal_cost(ctx, sur, _item(12, 0.3, 100), np.linspace(-6, 6, 1024), (-2.0, 2.0),
                      (16, 24, 32, 48, 64, 96, 128, 192, 256))
    for row in r["rows"]:
        print(row)
    print("solves to 1e-4 (and every larger budget):", r["solves_to_tol"], "first within 1e-4:",
          r["first_within_tol"], "dense", r["dense_solves"])
    s_u, s_g = r["solves_to_tol"]["uniform"], r["solves_to_tol"]["guided"]
    assert s_u is not None and s_g is not None and s_g <= s_u
    big = [row for row in r["rows"] if row["solves"] >= min(s_u, s_g)]
    assert len(big) >= 3 and all(row["guided"] < row["uniform"] for row in big)
    assert all(row["guided_solves"] == row["uniform_solves"] == row["solves"] for row in r["rows"])
