"""Whole-face contacts (the DENSE self-energy case of Section 3.1.2): GPU solve through the C ABI
against the dense oracle with face self-energies, and closed forms.

Tolerance: max relative error per energy and output vector (max_i |x_i - y_i| / max_i |y_i|;
for T: |dT| / max(T, 1e-12)) <= 1e-10.  The FP64 paths (precision 0 and 1) eliminate cluster
blocks without pivoting across them in FP64, which at eta = 1e-8 loses digits in band whatever the
contacts; their dense-contact code is checked at eta = 0.05, where the pivot blocks stay well
conditioned.
"""
import numpy as np
import pytest
import torch

import synth
import oracle
import paper_1702_05167_amd as pkg

pytestmark = pytest.mark.gpu

KW = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1)
ALL = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS | pkg.HSC_SPECTRAL_LR
TOL = {0: 1e-10, 1: 1e-10, 2: 1e-10, 3: 1e-10}
ETA = {0: 0.05, 1: 0.05, 2: 1e-8, 3: 1e-8}
E_MIX = np.array([-4.6, -2.1, -0.7, 0.4, 1.8, 3.3, 5.2])


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def gpu(ctx, dev, energies, leaf, precision, want=ALL, dense=True, **kw):
    tree = pkg.Tree.from_device(dev, leaf_side=leaf, dense=dense)
    out = pkg.solve(ctx, tree, torch.tensor(np.asarray(energies, float), device=ctx.torch_device), want=want,
                    precision=precision, **{**KW, **kw})
    res = {k: v.cpu().numpy() for k, v in out.items()}
    if "spectral" in res:
        res["a_l"], res["a_r"] = res["spectral"][:, 0], res["spectral"][:, 1]
    return res


def check(g, ref, energies, tol, keys=("gr", "gl", "a_l", "a_r")):
    worst = 0.0
    for e in range(len(energies)):
        for k in keys:
            err = rel(g[k][e], ref[k][e])
            worst = max(worst, err)
            assert err <= tol, (k, energies[e], err)
        if "trans" in g:
            err = abs(g["trans"][e] - ref["trans"][e]) / max(ref["trans"][e], 1e-12)
            worst = max(worst, err)
            assert err <= tol, ("trans", energies[e], err, g["trans"][e], ref["trans"][e])
    assert (g["status"] == 0).all(), g["status"]
    return worst


def _disordered(shape, seed, sigma=0.3):
    n = shape[0] * shape[1] * shape[2]
    return synth.cuboid(*shape, onsite=np.random.default_rng(seed).normal(0.0, sigma, n))


@pytest.mark.parametrize("precision", [0, 1, 2, 3])
def test_dense_cube8_against_oracle(ctx, precision):
    dev = _disordered((8, 8, 8), 11)
    print(f"[dense cube8 precision {precision}]", flush=True)
    kw = {**KW, "eta": ETA[precision]}
    g = gpu(ctx, dev, E_MIX, 3, precision, eta=kw["eta"])
    ref = oracle.dense.solve(dev, E_MIX, dense=True, **kw)
    print("dense cube8 precision", precision, "worst", check(g, ref, E_MIX, TOL[precision]))


@pytest.mark.parametrize("shape,leaf", [((2, 5, 4), 2), ((3, 4, 5), 2), ((4, 6, 3), 2), ((5, 4, 4), 2),
                                        ((9, 5, 1), 2), ((6, 3, 7), 2), ((11, 4, 4), 3)])
def test_dense_shapes_against_oracle(ctx, shape, leaf):
    # two and three planes (the left face heads a chain), four (right face a leaf), five and more
    # (both faces above their halves), a 2D device, ragged faces
    dev = _disordered(shape, 5)
    print(f"[dense shape {shape} leaf {leaf}]", flush=True)
    g = gpu(ctx, dev, E_MIX, leaf, 3)
    ref = oracle.dense.solve(dev, E_MIX, dense=True, **KW)
    print("dense", shape, "worst", check(g, ref, E_MIX, TOL[3]))


def test_dense_cube12_against_oracle(ctx):
    dev = _disordered((12, 12, 12), 21)
    E = np.array([-3.9, -1.3, 0.25, 2.05, 4.4])
    print("[dense cube12]", flush=True)
    g = gpu(ctx, dev, E, 4, 3, batch=3)
    ref = oracle.dense.solve(dev, E, dense=True, **KW)
    print("dense cube12 worst", check(g, ref, E, TOL[3]))


def test_dense_transmission_only_and_graph(ctx):
    # the transmission-only plan (right channel extracted on the left path) and graph replay give
    # the same T as the full solve
    dev = _disordered((7, 6, 5), 2)
    full = gpu(ctx, dev, E_MIX, 3, 3)
    t_only = gpu(ctx, dev, E_MIX, 3, 3, want=pkg.HSC_TRANS, graph=1, batch=4)
    assert np.allclose(t_only["trans"], full["trans"], rtol=1e-12, atol=1e-14)
    gr_gl = gpu(ctx, dev, E_MIX, 3, 2, want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS)
    ref = oracle.dense.solve(dev, E_MIX, dense=True, **KW)
    check(gr_gl, ref, E_MIX, TOL[2], keys=("gr", "gl"))


def test_dense_clean_wire_counts_open_modes(ctx):
    # clean device with the lead's own parameters: T(E) = number of open transverse modes
    dev = synth.cuboid(9, 6, 5)
    lam = []
    for p in range(1, 7):
        for q in range(1, 6):
            lam.append(-2.0 * (np.cos(np.pi * p / 7) + np.cos(np.pi * q / 6)))
    lam = np.array(lam)
    E = [e for e in np.linspace(-6.4, 6.4, 41) if np.abs(np.concatenate([lam - 2, lam + 2]) - e).min() > 0.05]
    g = gpu(ctx, dev, E, 3, 3, want=pkg.HSC_TRANS, eta=1e-12)
    count = np.array([np.sum(np.abs(e - lam) < 2.0) for e in E])
    assert np.abs(g["trans"] - count).max() < 1e-6, np.c_[E, g["trans"], count]


def test_dense_chain_equals_per_site_leads(ctx):
    # one-site faces: the whole-face lead is the 1D chain lead
    dev = synth.chain(13, onsite=np.random.default_rng(4).normal(0, 0.3, 13))
    a = gpu(ctx, dev, E_MIX, 2, 3, dense=False)
    b = gpu(ctx, dev, E_MIX, 2, 3, dense=True)
    for k in ("gr", "gl", "a_l", "a_r"):
        assert rel(b[k], a[k]) < 1e-13, k
    assert np.allclose(b["trans"], a["trans"], rtol=1e-12, atol=1e-15)


def test_dense_batch_solves_each_device(ctx):
    devs = [_disordered((6, 4, 4), 31), _disordered((5, 5, 3), 32)]
    trees = [pkg.Tree.from_device(d, leaf_side=2, dense=True) for d in devs]
    E = torch.tensor(E_MIX, device=ctx.torch_device)
    outs = pkg.solve_batch(ctx, trees, E, want=ALL, precision=3, **KW)
    for d, o in zip(devs, outs):
        res = {k: v.cpu().numpy() for k, v in o.items()}
        res["a_l"], res["a_r"] = res["spectral"][:, 0], res["spectral"][:, 1]
        check(res, oracle.dense.solve(d, E_MIX, dense=True, **KW), E_MIX, TOL[3])


def test_dense_guard_rejected(ctx):
    dev = _disordered((6, 4, 4), 1)
    with pytest.raises(pkg.hsc.HscError):
        gpu(ctx, dev, E_MIX[:2], 2, 1, guard_tau=100.0)


@pytest.mark.parametrize("precision,slices", [(2, 0), (3, 0), (3, 15)])
def test_dense_cube32_golden_benchmark_configuration(ctx, precision, slices):
    # the 32^3 benchmark cube with whole-face contacts, in the benchmark's launch configuration
    # (3D nested dissection, leaves <= 8, batches of 16, tuned tiles), against the slab recursion
    # with the dense face blocks at four energies of the 256-point grid (all sites' diagonals were
    # computed there; 68 are stored)
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "dense32_rgf.json")))
    E, sites = np.array(gold["energies"]), np.array(gold["sites"])
    ref = {"gr": np.array(gold["gr_re"]) + 1j * np.array(gold["gr_im"]),
           "gl": np.array(gold["gl_re"]) + 1j * np.array(gold["gl_im"]),
           "a_l": np.array(gold["a_l"]), "a_r": np.array(gold["a_r"]), "trans": np.array(gold["trans"])}
    print(f"[dense cube32 golden precision {precision} slices {slices}]", flush=True)
    Ep = np.tile(E, 4)                 # one batch of 16
    g = gpu(ctx, synth.config1_device(), Ep, 8, precision, tune=1, batch=16, slices=slices)
    gs = {k: g[k][:4, sites] for k in ("gr", "gl", "a_l", "a_r")}
    gs["trans"], gs["status"] = g["trans"][:4], g["status"][:4]
    print("dense 32^3 golden worst", check(gs, ref, E, TOL[precision]))
    for k in ("gr", "gl", "trans"):    # every quarter of the batch solves the same energies
        assert np.array_equal(g[k][:4], g[k][4:8]) and np.array_equal(g[k][:4], g[k][12:]), k
