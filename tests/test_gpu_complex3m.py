"""The solve with three real products per complex multiply-add (opts.complex3m) against the oracle."""
import numpy as np
import pytest

import synth
import oracle
import paper_1702_05167_amd as pkg
from test_gpu_parity import (ALL, GUARD, IN_BAND, KW, TOL, _golden32_check, _modes, _trilayer_check, check_all,
                             gpu, rel, t_rel)

pytestmark = pytest.mark.gpu


def test_3m_clean_cuboid_modes(ctx):
    nx, ny, nz = 7, 5, 4
    g = gpu(ctx, synth.cuboid(nx, ny, nz), np.array([-4.1, -1.2, 0.3, 2.2]), 2, complex3m=1, **GUARD)
    for e, en in enumerate([-4.1, -1.2, 0.3, 2.2]):
        gr, al, ar, T = _modes(nx, ny, nz, en)
        assert max(rel(g["gr"][e], gr), rel(g["a_l"][e], al), rel(g["a_r"][e], ar), t_rel(g["trans"][e], T)) <= TOL


def test_3m_config0_all_energies_guarded(ctx):
    dev = synth.config0_device()
    E = synth.energy_grid(-5.0, 5.0, 16)
    g = gpu(ctx, dev, E, 4, complex3m=1, **GUARD)
    print("worst", check_all(g, oracle.dense.solve(dev, E, **KW), E))


def test_3m_cube32_golden_in_band_transverse_tree(ctx):
    print("worst", _golden32_check(ctx, IN_BAND, leaf=4, transverse=True, precision=0, complex3m=1))


def test_3m_trilayer_golden_guarded(ctx):
    print("worst", _trilayer_check(ctx, leaf=8, precision=0, guard_tau=30.0, guard_rounds=8, complex3m=1))


def test_3m_tuned_equals_untuned(ctx):
    dev = synth.config1_device(n_side=16)
    tree = pkg.Tree.from_device(dev, leaf_side=4, transverse=True)
    E = np.array([-1.4, 0.6, 1.7])
    a = pkg.solve(ctx, tree, E, want=ALL, precision=0, complex3m=1, **KW)
    b = pkg.solve(ctx, tree, E, want=ALL, precision=0, complex3m=1, tune=1, **KW)
    for k in a:
        x, y = a[k].cpu().numpy(), b[k].cpu().numpy()
        assert np.allclose(y, x, rtol=1e-12, atol=1e-12 * np.abs(x).max()), k
