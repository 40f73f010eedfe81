"""Multi-device batches (forest of uneven devices) and graph replay, through the C ABI."""
import numpy as np
import pytest
import torch

import synth
import oracle
import paper_1702_05167_amd as pkg
from oracle.negf import gamma_of, sigma_lead

pytestmark = pytest.mark.gpu

KW = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1)
ALL = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS | pkg.HSC_SPECTRAL_LR


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def _uneven(seed=3):
    rng = np.random.default_rng(seed)
    devs = []
    for k, (nx, ny, nz) in enumerate([(6, 5, 4), (9, 7, 6), (5, 8, 7), (7, 4, 9)]):
        devs.append(synth.cuboid(nx, ny, nz, onsite=rng.normal(0, 0.3, nx * ny * nz), name=f"u{k}"))
    return devs


def _np(o):
    return {k: v.cpu().numpy() for k, v in o.items()}


def test_forest_matches_dense_oracle_per_device(ctx):
    devs = _uneven()
    trees = [pkg.Tree.from_device(d, leaf_side=3) for d in devs]
    E = np.array([-1.7, -0.6, 0.05, 0.9, 1.8])
    outs = pkg.solve_batch(ctx, trees, E, want=ALL, **KW)
    for d, o in zip(devs, outs):
        g = _np(o)
        ref = oracle.dense.solve(d, E, **KW)
        for e in range(len(E)):
            assert rel(g["gr"][e], ref["gr"][e]) <= 1e-10
            assert rel(g["gl"][e], ref["gl"][e]) <= 1e-10
            assert rel(g["spectral"][e, 0], ref["a_l"][e]) <= 1e-10
            assert rel(g["spectral"][e, 1], ref["a_r"][e]) <= 1e-10
            assert abs(g["trans"][e] - ref["trans"][e]) <= 1e-10 * max(ref["trans"][e], 1e-12)
        assert (g["status"] == 0).all()


def test_forest_out_of_band_double_double(ctx):
    # uneven devices in one forest at energies outside the lead band, where only the double-double
    # solve keeps every block product exact enough (no guard)
    devs = _uneven(11)
    trees = [pkg.Tree.from_device(d, leaf_side=3) for d in devs]
    E = np.array([-4.6, -3.1, -2.3, 2.45, 3.7, 5.2])
    outs = pkg.solve_batch(ctx, trees, E, want=ALL, precision=2, **KW)
    worst = 0.0
    for d, o in zip(devs, outs):
        g = _np(o)
        ref = oracle.dense.solve(d, E, **KW)
        for e in range(len(E)):
            errs = (rel(g["gr"][e], ref["gr"][e]), rel(g["gl"][e], ref["gl"][e]),
                    rel(g["spectral"][e, 0], ref["a_l"][e]), rel(g["spectral"][e, 1], ref["a_r"][e]),
                    abs(g["trans"][e] - ref["trans"][e]) / max(ref["trans"][e], 1e-12))
            worst = max(worst, max(errs))
            assert max(errs) <= 1e-10, (d.name, E[e], errs)
        assert (g["status"] == 0).all()
    print("forest out of band, double-double worst", worst)


@pytest.mark.parametrize("want", [ALL, pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS])
def test_forest_equals_single_device_solves(ctx, want):
    devs = _uneven(5)
    trees = [pkg.Tree.from_device(d, leaf_side=3) for d in devs]
    E = torch.linspace(-5, 5, 11, dtype=torch.float64, device="cuda")
    outs = pkg.solve_batch(ctx, trees, E, want=want, batch=4, **KW)
    for t, o in zip(trees, outs):
        s = _np(pkg.solve(ctx, t, E, want=want, batch=4, **KW))
        for k in s:
            a, b = _np(o)[k], s[k]
            assert np.allclose(a, b, rtol=1e-13, atol=1e-13 * np.abs(b).max()), k


def test_batch_with_different_energies_solves_each_device(ctx):
    devs = _uneven(7)[:2]
    trees = [pkg.Tree.from_device(d, leaf_side=3) for d in devs]
    Es = [np.array([-1.1, 0.4]), np.array([0.3, 1.2, 1.9])]
    outs = pkg.solve_batch(ctx, trees, Es, **KW)
    for t, o, E in zip(trees, outs, Es):
        s = _np(pkg.solve(ctx, t, E, **KW))
        for k in ("gr", "gl", "trans"):
            assert np.array_equal(_np(o)[k], s[k])


@pytest.mark.parametrize("want", [ALL, pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS, pkg.HSC_DIAG_GR])
def test_graph_replay_equals_step_launches(ctx, want):
    dev = synth.config0_device()
    tree = pkg.Tree.from_device(dev, leaf_side=4)
    for E in (np.linspace(-4.5, 4.5, 13), np.array([0.3, -1.2, 2.2, 0.7, -0.1])):
        a = _np(pkg.solve(ctx, tree, E, want=want, batch=4, **KW))
        for rep in range(3):                 # replays with eager work and syncs in between
            b = _np(pkg.solve(ctx, tree, E, want=want, batch=4, graph=1, **KW))
            for k in a:
                assert np.array_equal(a[k], b[k]), (k, rep)
            torch.cuda.synchronize()


def test_graph_forest(ctx):
    devs = _uneven(11)
    trees = [pkg.Tree.from_device(d, leaf_side=3) for d in devs]
    E = np.linspace(-1.9, 1.9, 9)
    a = pkg.solve_batch(ctx, trees, E, want=ALL, batch=4, **KW)
    b = pkg.solve_batch(ctx, trees, E, want=ALL, batch=4, graph=1, **KW)
    for oa, ob in zip(a, b):
        for k in oa:
            assert torch.equal(oa[k], ob[k]), k


def test_uneven_config2_subset_invariants(ctx):
    # four of the 64 uneven devices (sides 16..48), transverse trees, in-band energies
    devs = synth.config2_devices(which=[1, 2, 6, 7])
    trees = [pkg.Tree.from_device(d, leaf_side=4, transverse=True) for d in devs]
    E = np.array([-1.6, -0.45, 0.1, 1.25])
    outs = pkg.solve_batch(ctx, trees, E, want=ALL, precision=0, **KW)
    for d, o in zip(devs, outs):
        g = _np(o)
        assert (g["status"] == 0).all()
        left, right = d.contacts[0].sites, d.contacts[1].sites
        for e, en in enumerate(E):
            gam = gamma_of(sigma_lead(en + 1e-8j, 0.0, -1.0, -1.0))
            t_lr = gam * g["spectral"][e, 1][left].sum()
            t_rl = gam * g["spectral"][e, 0][right].sum()
            assert abs(t_lr - t_rl) <= 1e-9 * t_lr
            assert abs(g["trans"][e] - t_lr) <= 1e-12 * t_lr
            assert (g["gr"][e].imag <= 1e-10 * np.abs(g["gr"][e]).max()).all()
            assert (g["gl"][e].imag >= -1e-10 * np.abs(g["gl"][e]).max()).all()


def test_tuned_plan_equals_default(ctx):
    # the tuner only changes tile shapes; the 16x16x4 shapes sum in the same order as the default,
    # the 4x4x4 shape agrees to rounding
    dev = synth.config1_device(n_side=16)
    tree = pkg.Tree.from_device(dev, leaf_side=4, transverse=True)
    E = np.array([-1.4, -0.2, 0.6, 1.7, 3.1])
    a = _np(pkg.solve(ctx, tree, E, want=ALL, precision=0, **KW))
    b = _np(pkg.solve(ctx, tree, E, want=ALL, precision=0, tune=1, **KW))
    c = _np(pkg.solve(ctx, tree, E, want=ALL, precision=0, tune=1, graph=1, **KW))
    for k in a:
        for x in (b[k], c[k]):
            assert np.allclose(x, a[k], rtol=1e-12, atol=1e-12 * np.abs(a[k]).max()), k


@pytest.mark.parametrize("precision,slices", [(2, 0), (3, 0), (3, 15)])
def test_config2_devices_against_stored_oracle(ctx, precision, slices):
    # four of the 64 uneven cuboids (the smallest, 16 x 20 x 16, to the largest, 48 x 43 x 47 =
    # 97,008 sites) in one hsc_solve_batch call on 3D trees with leaves <= 8, at two energies of the
    # 128-point grid in the lead band and two outside it, against refined sparse-LU rows of G^r
    # at 66 sites per device (tests/golden/make_config2.py)
    import json
    import os
    gold = json.load(open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                                       "config2_sampled.json")))
    E = np.array(gold["energies"])
    ids = [d["device"] for d in gold["devices"]]
    devs = [synth.config2_devices(which=[i])[0] for i in ids]      # in the stored order
    trees = [pkg.Tree.from_device(d, leaf_side=8) for d in devs]
    print(f"[config2 precision {precision} slices {slices}]", flush=True)
    outs = pkg.solve_batch(ctx, trees, torch.tensor(E, device=ctx.torch_device), precision=precision,
                           want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS, slices=slices, **KW)
    worst = 0.0
    for d, o in zip(gold["devices"], outs):
        sites = np.array(d["sites"])
        ne = len(E)
        ref_gr = (np.array(d["gr_re"]) + 1j * np.array(d["gr_im"])).reshape(ne, -1)
        ref_gl = (np.array(d["gl_re"]) + 1j * np.array(d["gl_im"])).reshape(ne, -1)
        gr = o["gr"].cpu().numpy()[:, sites]
        gl = o["gl"].cpu().numpy()[:, sites]
        tr = o["trans"].cpu().numpy()
        assert (o["status"].cpu().numpy() == 0).all()
        for e in range(ne):
            errs = (rel(gr[e], ref_gr[e]), rel(gl[e], ref_gl[e]),
                    abs(tr[e] - d["trans"][e]) / max(d["trans"][e], 1e-12))
            worst = max(worst, *errs)
            print("device", d["device"], d["sides"], "E", E[e], errs)
            assert max(errs) <= 1e-10, (d["device"], E[e], errs)
    print("config2 worst", worst)
