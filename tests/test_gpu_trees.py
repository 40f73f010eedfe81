"""Other trees (Section 2.2: any cluster tree whose separators separate; a chain of slabs is the
recursive Green's function of Section 2.1; the DNA study's customised partitions) and graph nested
dissection for unstructured H: GPU solve through the C ABI against the dense oracle.

Tolerance: max relative error per energy and output vector <= 1e-10 (T: |dT| / max(T, 1e-12)).
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


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def run(ctx, dev, tree, E, precision=3, eta=1e-8):
    out = pkg.solve(ctx, tree, torch.tensor(E, device=ctx.torch_device), want=ALL, precision=precision,
                    **{**KW, "eta": eta})
    g = {k: v.cpu().numpy() for k, v in out.items()}
    g["a_l"], g["a_r"] = g["spectral"][:, 0], g["spectral"][:, 1]
    ref = oracle.dense.solve(dev, E, **{**KW, "eta": eta})
    worst = 0.0
    for e in range(len(E)):
        for k in ("gr", "gl", "a_l", "a_r"):
            err = rel(g[k][e], ref[k][e])
            worst = max(worst, err)
            assert err <= 1e-10, (k, E[e], err)
        err = abs(g["trans"][e] - ref["trans"][e]) / max(ref["trans"][e], 1e-12)
        worst = max(worst, err)
        assert err <= 1e-10, ("trans", E[e], err)
    assert (g["status"] == 0).all()
    return worst, g


@pytest.mark.parametrize("n,k,leaf", [(600, 6, 40), (900, 8, 60), (300, 4, 10)])
def test_graph_dissection_unstructured(ctx, n, k, leaf):
    dev = synth.random_graph_device(n, k, seed=n + k)
    E = np.array([-4.1, -1.9, -0.6, 0.7, 2.2, 4.8])
    print(f"[graph nd n={n} k={k}]", flush=True)
    w, _ = run(ctx, dev, pkg.Tree.from_device(dev, leaf_side=leaf, graph=True), E)
    print("graph nd", n, k, "worst", w)


def test_graph_dissection_fp64_path(ctx):
    dev = synth.random_graph_device(600, 6, seed=3)
    E = np.array([-2.5, -0.3, 1.4])
    w, _ = run(ctx, dev, pkg.Tree.from_device(dev, leaf_side=40, graph=True), E, precision=0, eta=0.05)
    print("graph nd fp64 worst", w)


def test_graph_dissection_cube_matches_geometric(ctx):
    dev = synth.cuboid(10, 9, 8, onsite=np.random.default_rng(4).normal(0, 0.3, 720))
    E = np.array([-3.3, -0.9, 0.15, 1.6, 4.2])
    wg, g = run(ctx, dev, pkg.Tree.from_device(dev, leaf_side=60, graph=True), E)
    wd, d = run(ctx, dev, pkg.Tree.from_device(dev, leaf_side=4), E)
    for key in ("gr", "gl", "trans"):
        assert rel(g[key], d[key]) < 1e-10, key
    print("graph vs geometric cube worst", wg, wd)


def test_slab_chain_is_rgf(ctx):
    # the degenerate (chain) tree makes the method the slab recursion: same values as the dense
    # oracle and as oracle.rgf
    dev = synth.cuboid(9, 5, 4, onsite=np.random.default_rng(5).normal(0, 0.3, 180))
    E = np.array([-1.7, -0.4, 0.9, 1.8])
    w, g = run(ctx, dev, pkg.Tree.slab_chain(dev), E)
    r = oracle.rgf.solve(dev, E, **KW)
    assert rel(g["gr"], r["gr"]) < 1e-10 and rel(g["trans"], r["trans"]) < 1e-10
    print("slab chain worst", w)


@pytest.mark.parametrize("partition", ["pairs_chain", "two_pair_chain", "custom_nd", "geometric"])
def test_dna_ladder_partitions(ctx, partition):
    # dense base-pair blocks; partitions of the DNA study: one base pair per layer (RGF), two base
    # pairs per layer, a hand-made dissection over base pairs, and the geometric tree
    dev = synth.dna_ladder(11, 8, seed=2)
    E = np.array([-2.4, -1.1, -0.2, 0.6, 1.9])
    pair = dev.coords[:, 0].astype(np.int64)
    contacts = [(c.sites, c.lead_onsite, c.lead_hopping, c.coupling) for c in dev.contacts]
    args = (dev.n, dev.indptr, dev.indices, dev.values, contacts)
    if partition == "pairs_chain":
        tree = pkg.Tree.slab_chain(dev)
    elif partition == "two_pair_chain":
        layer = pair // 2
        nl = int(layer.max()) + 1
        tree = pkg.Tree.build_custom(*args, layer, list(range(1, nl)) + [-1])
    elif partition == "custom_nd":
        groups = {5: 0, 2: 1, 8: 2, 0: 3, 1: 3, 3: 4, 4: 4, 6: 5, 7: 5, 9: 6, 10: 6}
        tree = pkg.Tree.build_custom(*args, np.array([groups[p] for p in pair]), [-1, 0, 0, 1, 1, 2, 2])
    else:
        tree = pkg.Tree.from_device(dev, leaf_side=1)
    print(f"[dna {partition}]", flush=True)
    w, _ = run(ctx, dev, tree, E)
    print("dna", partition, "worst", w, "flops", tree.stats()["flops_per_energy"])
