"""Multi-orbital site blocks (b x b per site, the block structure of the paper's sp3d5s* nanowire
Hamiltonians, with random blocks): GPU solve through the C ABI against the dense oracle.

Tolerance as in the other parity tests: max relative error per energy and output vector <= 1e-10
(T: |dT| / max(T, 1e-12)); the FP64 path (precision 0) at eta = 0.05, where its unpivoted
elimination keeps its digits.
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
E = np.array([-5.2, -2.6, -1.1, 0.3, 1.7, 3.9, 6.4])


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def run(ctx, dev, leaf, precision, eta=1e-8, **kw):
    tree = pkg.Tree.from_device(dev, leaf_side=leaf)
    out = pkg.solve(ctx, tree, torch.tensor(E, device=ctx.torch_device), want=ALL, precision=precision,
                    **{**KW, "eta": eta}, **kw)
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
    return worst


@pytest.mark.parametrize("shape,b,leaf", [((6, 4, 3), 4, 2), ((7, 3, 3), 10, 2), ((5, 5, 5), 2, 2),
                                          ((9, 2, 2), 10, 1), ((4, 4, 4), 6, 3)])
def test_orbital_blocks_against_oracle(ctx, shape, b, leaf):
    dev = synth.orbital_cuboid(*shape, b, seed=7)
    print(f"[orbitals {shape} b={b}]", flush=True)
    print("orbitals", shape, b, "precision 3 worst", run(ctx, dev, leaf, 3))


def test_orbital_blocks_fp64_path(ctx):
    dev = synth.orbital_cuboid(6, 4, 3, 4, seed=8)
    print("orbitals fp64 worst", run(ctx, dev, 2, 0, eta=0.05))


def test_ten_orbital_wire_symmetries(ctx):
    # a 10-orbital wire (64 x 4 x 4 sites, 10,240 unknowns): transmission reciprocity between the two
    # channels, current conservation of the spectral functions, and the sum rule at the broadened
    # energies -2 Im G^r >= A_L + A_R (the rest is the eta broadening, positive)
    dev = synth.orbital_cuboid(64, 4, 4, 10, seed=9)
    tree = pkg.Tree.from_device(dev, leaf_side=2)
    out = pkg.solve(ctx, tree, torch.tensor(E, device=ctx.torch_device), want=ALL, precision=3, **KW)
    g = {k: v.cpu().numpy() for k, v in out.items()}
    a_l, a_r = g["spectral"][:, 0], g["spectral"][:, 1]
    left = dev.contacts[0].sites
    right = dev.contacts[1].sites
    gam = -2.0 * np.imag(oracle.negf.sigma_lead(E + 1e-8j, 0.0, -1.0, -1.0))
    t_lr = gam * a_r[:, left].sum(1)
    t_rl = gam * a_l[:, right].sum(1)
    assert np.allclose(t_lr, g["trans"], rtol=1e-10, atol=1e-14)
    assert np.allclose(t_rl, t_lr, rtol=1e-9, atol=1e-12)
    assert (-2 * g["gr"].imag - (a_l + a_r) >= -1e-9 * np.abs(g["gr"]).max()).all()
    assert (g["status"] == 0).all()
