"""Concurrent batches (`hsc_solve_opts.streams`): the batches of one call round-robin on several
streams of the context, each with its own plan.  Every slot of a batch computes what it computes on
one stream, so the outputs must be bit-identical to the one-stream call; the call must stay ordered
on the context's stream (a context on a stream of its own synchronises only that stream)."""
import numpy as np
import pytest
import torch

import synth
import paper_1702_05167_amd as pkg
import paper_1702_05167_amd.hsc as H

pytestmark = pytest.mark.gpu

WANT = pkg.HSC_DIAG_GR | pkg.HSC_DIAG_GL | pkg.HSC_TRANS
KW = dict(eta=1e-8, kT=0.025, mu_L=0.1, mu_R=-0.1, want=WANT)


def _device():
    return synth.cuboid(10, 9, 8, onsite=np.random.default_rng(21).uniform(-0.5, 0.5, 720))


def _same(a, b):
    for k in ("gr", "gl", "trans", "status"):
        assert torch.equal(a[k], b[k]), k


@pytest.mark.parametrize("precision,streams", [(3, 4), (3, 3), (0, 2)])
def test_streams_match_one_stream(precision, streams):
    # 30 energies in batches of 4 (the last one partial), on a context with a stream of its own
    s = torch.cuda.Stream()
    ctx = pkg.Context(0, stream=s)
    try:
        tree = pkg.Tree.from_device(_device(), leaf_side=4)
        E = torch.tensor(np.linspace(-5.0, 5.0, 30), dtype=torch.float64, device=ctx.torch_device)
        torch.cuda.synchronize()
        print(f"[streams {streams} precision {precision}]", flush=True)
        one = pkg.solve(ctx, tree, E, batch=4, precision=precision, **KW)
        many = pkg.solve(ctx, tree, E, batch=4, precision=precision, streams=streams, **KW)
        if precision == 3:
            assert int(many["status"].abs().max()) == 0
        _same(one, many)
        # a second call reuses the plans of every stream
        again = pkg.solve(ctx, tree, E, batch=4, precision=precision, streams=streams, **KW)
        _same(one, again)
    finally:
        ctx.close()


def test_streams_with_graphs_and_a_potential(ctx):
    tree = pkg.Tree.from_device(_device(), leaf_side=4)
    E = torch.tensor(np.linspace(-4.0, 4.0, 12), dtype=torch.float64, device=ctx.torch_device)
    pot = torch.tensor(np.random.default_rng(3).normal(0, 0.1, tree.n), device=ctx.torch_device)
    one = pkg.solve(ctx, tree, E, batch=3, graph=1, potential=pot, **KW)
    many = pkg.solve(ctx, tree, E, batch=3, graph=1, potential=pot, streams=4, **KW)
    _same(one, many)
    # without the potential again: every stream's plan clears it
    zero = pkg.solve(ctx, tree, E, batch=3, **KW)
    many0 = pkg.solve(ctx, tree, E, batch=3, streams=4, **KW)
    _same(zero, many0)


def test_streams_in_a_forest(ctx):
    trees = [pkg.Tree.from_device(synth.cuboid(n, 6, 5), leaf_side=4) for n in (6, 9, 7)]
    E = np.linspace(-3.0, 3.0, 10)
    one = pkg.solve_batch(ctx, trees, E, batch=2, **KW)
    many = pkg.solve_batch(ctx, trees, E, batch=2, streams=3, **KW)
    for a, b in zip(one, many):
        _same(a, b)


def test_streams_out_of_range(ctx):
    tree = pkg.Tree.from_device(synth.cuboid(4, 4, 4), leaf_side=4)
    E = torch.zeros(4, dtype=torch.float64, device=ctx.torch_device)
    for k in (-1, 9):
        with pytest.raises(H.HscError):
            pkg.solve(ctx, tree, E, batch=2, streams=k, **KW)


def test_streams_fall_back_to_one_with_profiling_and_the_guard(ctx):
    # launch timing and the growth guard run on the context's stream alone; the option is accepted
    # and the results are those of one stream
    tree = pkg.Tree.from_device(_device(), leaf_side=4)
    E = torch.tensor(np.linspace(-4.0, 4.0, 8), dtype=torch.float64, device=ctx.torch_device)
    one = pkg.solve(ctx, tree, E, batch=2, **KW)
    ctx.profile(True)
    try:
        prof = pkg.solve(ctx, tree, E, batch=2, streams=4, **KW)
        assert sum(v["launches"] for v in ctx.profile_read().values()) > 0
    finally:
        ctx.profile(False)
    _same(one, prof)
    guarded = pkg.solve(ctx, tree, E, batch=2, streams=4, guard=True, guard_tau=1e30, **KW)
    _same(one, guarded)
