"""Off-diagonal entries on the bonds of H (the desired off-diagonal entries of G^r and G^<;
bond currents follow from G^<_ij H_ji): GPU solve through the C ABI (hsc_solve_ex) against the
dense oracle, and the continuity identity on the GPU's own outputs.

Tolerance: max_b |x_b - y_b| / max_b |y_b| <= 1e-10 per energy and output; the FP64 path
(precision 0) at eta = 0.05 (its unpivoted elimination keeps its digits there).
"""
import numpy as np
import pytest
import torch

import synth
import oracle
import paper_1702_05167_amd as pkg

pytestmark = pytest.mark.gpu

KW = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1)
BONDS = pkg.HSC_BOND_GR | pkg.HSC_BOND_GL
E = np.array([-4.4, -1.6, -0.35, 0.8, 2.9, 5.3])


def rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def gpu(ctx, dev, leaf, precision, want, dense=False, transverse=False, **kw):
    tree = pkg.Tree.from_device(dev, leaf_side=leaf, dense=dense, transverse=transverse)
    out = pkg.solve(ctx, tree, torch.tensor(E, device=ctx.torch_device), want=want, precision=precision,
                    **{**KW, **kw})
    return tree, {k: v.cpu().numpy() for k, v in out.items()}


def check(ctx, dev, leaf, precision, want=BONDS | pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL, dense=False, eta=1e-8,
          **kw):
    tree, g = gpu(ctx, dev, leaf, precision, want, dense=dense, eta=eta, **kw)
    pairs = tree.bonds()
    ref = oracle.dense.bonds(dev, E, eta, KW["kT"], KW["mu_L"], KW["mu_R"], pairs, dense=dense)
    worst = 0.0
    for e in range(len(E)):
        for key, rk in (("bond_gr", "gr"), ("bond_gl", "gl")):
            if key in g:
                err = rel(g[key][e], ref[rk][e])
                worst = max(worst, err)
                assert err <= 1e-10, (key, E[e], err)
    assert (g["status"] == 0).all()
    return worst, g


def _dis(shape, seed):
    return synth.cuboid(*shape, onsite=np.random.default_rng(seed).normal(0, 0.3, int(np.prod(shape))))


@pytest.mark.parametrize("precision", [0, 2, 3])
def test_bonds_cube8(ctx, precision):
    # 3D tree, leaves <= 4: bonds inside leaves, inside separators and between clusters
    print(f"[bonds cube8 precision {precision}]", flush=True)
    w, _ = check(ctx, _dis((8, 8, 8), 1), 4, precision, eta=0.05 if precision == 0 else 1e-8)
    print("bonds cube8 precision", precision, "worst", w)


@pytest.mark.parametrize("case", ["transverse", "dense", "orbitals", "spectral", "bond_gl_only"])
def test_bonds_variants(ctx, case):
    print(f"[bonds {case}]", flush=True)
    if case == "transverse":
        w, _ = check(ctx, _dis((9, 6, 5), 2), 3, 3, transverse=True)
    elif case == "dense":
        w, _ = check(ctx, _dis((7, 5, 4), 3), 2, 3, dense=True)
    elif case == "orbitals":
        w, _ = check(ctx, synth.orbital_cuboid(5, 3, 3, 4, seed=4), 2, 3)
    elif case == "spectral":
        # three lesser channels in one plan: A_L, A_R and the combined one for the bonds
        w, g = check(ctx, _dis((6, 5, 4), 5), 2, 2, want=BONDS | pkg.HSC_SPECTRAL_LR | pkg.HSC_TRANS)
        d = oracle.dense.solve(_dis((6, 5, 4), 5), E, **KW)
        assert rel(g["spectral"][:, 0], d["a_l"]) < 1e-10 and rel(g["spectral"][:, 1], d["a_r"]) < 1e-10
    else:
        w, _ = check(ctx, _dis((6, 5, 4), 6), 2, 3, want=pkg.HSC_BOND_GL)
    print("bonds", case, "worst", w)


def test_bond_currents_conserved(ctx):
    # on the GPU's own outputs: at every site without a lead,
    # sum_j (H_ij G^<_ji - G^<_ij H_ji) = 2 i eta G^<_ii
    dev = _dis((8, 6, 5), 7)
    eta = 1e-3
    tree, g = gpu(ctx, dev, 3, 3, BONDS | pkg.HSC_DIAG_GL, eta=eta)
    pairs = tree.bonds()
    h = dev.scipy_h().tocsr()
    hij = np.asarray(h[pairs[:, 0], pairs[:, 1]]).ravel()
    contact = np.zeros(dev.n, bool)
    for c in dev.contacts:
        contact[c.sites] = True
    for e in range(len(E)):
        gl = g["bond_gl"][e]
        # (H G^< - G^< H)_ii over the bonds at i: H_ij G^<_ji - G^<_ij H_ji with G^<_ji = -conj(G^<_ij)
        t = hij * (-np.conj(gl)) - gl * hij            # contribution to site i of bond (i, j)
        lhs = np.zeros(dev.n, np.complex128)
        np.add.at(lhs, pairs[:, 0], t)
        np.add.at(lhs, pairs[:, 1], -np.conj(t))      # the same bond seen from j
        rhs = 2j * eta * g["gl"][e]
        scale = np.abs(gl).max()
        assert np.abs((lhs - rhs)[~contact]).max() < 1e-11 * scale
    with pytest.raises(pkg.hsc.HscError):
        gpu(ctx, dev, 3, 1, BONDS, guard_tau=100.0)
