"""Argument checks of the C ABI on a GPU context: every bad call returns an error code, nothing runs."""
import ctypes as C

import numpy as np
import pytest
import torch

import synth
import paper_1702_05167_amd as pkg
import paper_1702_05167_amd.hsc as H

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def tree():
    return pkg.Tree.from_device(synth.cuboid(5, 4, 4), leaf_side=2)


def _code(fn):
    with pytest.raises(H.HscError) as e:
        fn()
    return e.value.code


@pytest.mark.parametrize("kw", [dict(want=0), dict(precision=4), dict(precision=-1), dict(complex3m=2), dict(eta=0.0),
                                dict(kT=-1.0), dict(guard=True, guard_tau=10.0, guard_rounds=-1)])
def test_solve_rejects_bad_options(ctx, tree, kw):
    assert _code(lambda: pkg.solve(ctx, tree, np.array([0.1, 0.2]), **kw)) == -1


def test_solve_rejects_clusters_beyond_the_dense_block_limit(ctx):
    # a 17^3 cube as one cluster (4913 sites > 4096, the largest block the batched inverses cover):
    # the plan is refused with HSC_E_ARG before anything is allocated or launched, the outputs
    # stay untouched
    tree = pkg.Tree.from_device(synth.cuboid(17, 17, 17), leaf_side=17)
    assert tree.stats()["max_cluster"] == 4913
    gr = torch.full((1, tree.n), 7.0, dtype=torch.complex128, device="cuda")
    for precision in (0, 2, 3):
        assert _code(lambda: pkg.solve(ctx, tree, np.array([0.3]), want=pkg.HSC_DIAG_GR, out={"gr": gr},
                                       precision=precision)) == -1
        assert b"dense-block limit" in H.lib().hsc_last_error()
    torch.cuda.synchronize()
    assert bool((gr == 7.0).all())


def test_solve_with_no_energies_is_a_no_op(ctx, tree):
    out = pkg.solve(ctx, tree, np.zeros(0))
    assert out["gr"].shape == (0, tree.n)


def test_batch_larger_than_energy_count(ctx, tree):
    a = pkg.solve(ctx, tree, np.array([-0.4, 0.9]), batch=64)
    b = pkg.solve(ctx, tree, np.array([-0.4, 0.9]), batch=1)
    for k in ("gr", "gl", "trans"):
        assert torch.equal(a[k], b[k])


def test_solve_rejects_missing_requested_output(ctx, tree):
    e = torch.tensor([0.3], dtype=torch.float64, device="cuda")
    opts = H.SolveOpts(1e-8, 0.025, 0.1, -0.1, pkg.HSC_DIAG_GR | pkg.HSC_TRANS, 0, 0.0, 0, 0, 0, 0, 0)
    gr = torch.empty((1, tree.n), dtype=torch.complex128, device="cuda")
    rc = H.lib().hsc_solve(ctx.h, tree.h, 1, H._dptr(e), C.byref(opts), H._dptr(gr), None, None, None, None, None)
    assert rc == -1 and b"trans" in H.lib().hsc_last_error()


def test_kernel_entry_points_reject_bad_arguments(ctx):
    A = torch.zeros((4, 4), dtype=torch.complex128, device="cuda")
    assert _code(lambda: H.kern_zgemm(ctx, 0, 0, 1.0, A, A, tile=9)) == -1
    assert _code(lambda: H.kern_zgemm(ctx, 3, 0, 1.0, A, A)) == -1
    X = torch.zeros((4, 4, 4), dtype=torch.float64, device="cuda")
    assert _code(lambda: H.kern_zgemm_dd(ctx, 0, 0, X, X, config=5)) == -1
    assert _code(lambda: H.kern_zinv_dd(ctx, X, matrix_cores=2)) == -1
    rc = H.lib().hsc_totals(ctx.h, 2, 10, None, None, None, None)
    assert rc == -1


@pytest.mark.parametrize("widths", [[4], [4, 0, 2], [4, 2000, 2]])
def test_network_rejects_bad_widths(ctx, widths):
    assert _code(lambda: pkg.MLP(ctx, widths)) == -1


def test_network_rejects_bad_training_options(ctx):
    net = pkg.MLP(ctx, [2, 3, 1])
    x = np.zeros((5, 2), np.float32)
    t = np.zeros((5, 1), np.float32)
    assert _code(lambda: net.train(x, t, steps=1, lr=0.0)) == -1
    assert _code(lambda: net.train(x, t, steps=1, beta1=1.0)) == -1
    with pytest.raises(ValueError):
        net.forward(np.zeros((3, 5), np.float32))
