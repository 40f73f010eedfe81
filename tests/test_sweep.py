"""Checkpointed energy sweeps (paper_1702_05167_amd/sweep.py) on the CPU with a stand-in solver: an
interrupted sweep resumes without solving finished chunks again, gives the outputs of an uninterrupted
one, and refuses a directory that holds another sweep."""
import types

import numpy as np
import pytest
import torch

from paper_1702_05167_amd.sweep import sweep

N_SITES = 5


class FakeSolver:
    def __init__(self, fail_at=None):
        self.calls = []
        self.fail_at = fail_at

    def __call__(self, ctx, tree, e, **kw):
        if self.fail_at is not None and len(self.calls) == self.fail_at:
            raise RuntimeError("interrupted")
        self.calls.append(e.clone())
        x = e.double()[:, None] * torch.arange(1, N_SITES + 1, dtype=torch.float64)
        return {"gr": torch.complex(x, -x), "gl": torch.complex(-x, x), "trans": e.double() ** 2,
                "status": torch.zeros(e.numel(), dtype=torch.int32)}


CTX = types.SimpleNamespace(torch_device="cpu")
TREE = types.SimpleNamespace(n=N_SITES)
E = np.linspace(-3.0, 3.0, 10)


def test_sweep_resumes_where_it_stopped(tmp_path):
    whole = sweep(CTX, TREE, E, tmp_path / "a", chunk=4, solve_fn=FakeSolver(), want=7)
    first = FakeSolver(fail_at=2)
    with pytest.raises(RuntimeError):
        sweep(CTX, TREE, E, tmp_path / "b", chunk=4, solve_fn=first, want=7)
    assert len(first.calls) == 2
    again = FakeSolver()
    out = sweep(CTX, TREE, E, tmp_path / "b", chunk=4, solve_fn=again, want=7)
    # only the third chunk (energies 8, 9) is solved again
    assert len(again.calls) == 1 and torch.equal(again.calls[0], torch.tensor(E[8:]))
    for k in ("gr", "gl", "trans", "status"):
        assert np.array_equal(out[k], whole[k]), k
    assert out["gr"].shape == (10, N_SITES) and out["gr"].dtype == np.complex128
    # a finished sweep loads entirely from disk
    done = FakeSolver()
    assert np.array_equal(sweep(CTX, TREE, E, tmp_path / "b", chunk=4, solve_fn=done, want=7)["trans"], whole["trans"])
    assert done.calls == []


def test_sweep_refuses_another_sweeps_directory(tmp_path):
    sweep(CTX, TREE, E, tmp_path, chunk=4, solve_fn=FakeSolver(), want=7)
    for kw in (dict(energies=E + 1e-3, chunk=4), dict(energies=E, chunk=5)):
        with pytest.raises(ValueError):
            sweep(CTX, TREE, kw["energies"], tmp_path, chunk=kw["chunk"], solve_fn=FakeSolver(), want=7)
    with pytest.raises(ValueError):
        sweep(CTX, TREE, E, tmp_path, chunk=4, solve_fn=FakeSolver(), want=3)
