"""A checkpointed sweep through the real solver: the outputs equal one solve of all energies, and a
second call reads them back from disk without solving."""
import numpy as np
import pytest
import torch

import synth
import paper_1702_05167_amd as pkg

pytestmark = pytest.mark.gpu


def test_sweep_matches_one_solve(ctx, tmp_path):
    dev = synth.cuboid(8, 7, 6, onsite=np.random.default_rng(31).uniform(-0.5, 0.5, 336))
    tree = pkg.Tree.from_device(dev, leaf_side=4)
    E = np.linspace(-4.5, 4.5, 11)
    kw = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, want=pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS,
              batch=4)
    ref = pkg.solve(ctx, tree, torch.tensor(E, device=ctx.torch_device), **kw)
    out = pkg.sweep(ctx, tree, E, tmp_path, chunk=4, **kw)
    # the last chunk (three energies) runs on a plan of three slots, the one-shot solve on four
    for k in ("gr", "gl", "trans"):
        r = ref[k].cpu().numpy()
        assert np.abs(out[k] - r).max() <= 1e-12 * np.abs(r).max(), k
    assert np.array_equal(out["status"], ref["status"].cpu().numpy())
    calls = []
    again = pkg.sweep(ctx, tree, E, tmp_path, chunk=4, solve_fn=lambda *a, **k: calls.append(1), **kw)
    assert calls == [] and np.array_equal(again["gl"], out["gl"])
