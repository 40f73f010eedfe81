"""The allocation-free double-double product (hsc_kern_zgemm_dd_noalloc) against the allocating
entry point (hsc_kern_zgemm_dd, config 3) through the C ABI: two calls in a row, the second smaller
(the static scratch keeps the first call's contents), and the size limit."""
import numpy as np
import pytest
import torch

import paper_1702_05167_amd.hsc as H

pytestmark = pytest.mark.gpu


def _dd_rand(rng, rows, cols):
    hi = rng.standard_normal((rows, cols, 2))
    lo = (rng.random((rows, cols, 2)) - 0.5) * np.spacing(np.abs(hi))
    out = np.empty((rows, cols, 4))
    out[..., 0], out[..., 1], out[..., 2], out[..., 3] = hi[..., 0], lo[..., 0], hi[..., 1], lo[..., 1]
    return out


@pytest.mark.parametrize("opA,opB,negate,beta", [(0, 0, 0, 1), (1, 1, 1, 0)])
def test_noalloc_product_matches_allocating_entry_point(ctx, opA, opB, negate, beta):
    rng = np.random.default_rng(31 + 2 * opA + opB)
    dev = ctx.torch_device
    for M, N, K in [(200, 150, 300), (70, 37, 45)]:      # the second call is smaller
        A = torch.tensor(_dd_rand(rng, *((M, K) if opA == 0 else (K, M))), device=dev)
        B = torch.tensor(_dd_rand(rng, *((K, N) if opB == 0 else (N, K))), device=dev)
        C = torch.tensor(_dd_rand(rng, M, N), device=dev) if beta else None
        ref = H.kern_zgemm_dd(ctx, opA, opB, A, B, negate=negate, beta=beta, C_=C, config=3)
        D = torch.full((M, N, 4), np.nan, dtype=torch.float64, device=dev)
        H.kern_zgemm_dd_noalloc(ctx, opA, opB, A, B, D, negate=negate, beta=beta, C_=C)
        assert torch.equal(D, ref), (M, N, K)


def test_noalloc_rejects_products_beyond_the_scratch(ctx):
    dev = ctx.torch_device
    A = torch.zeros((1024, 1024, 4), dtype=torch.float64, device=dev)
    D = torch.zeros((1024, 1024, 4), dtype=torch.float64, device=dev)
    with pytest.raises(H.HscError) as e:
        H.kern_zgemm_dd_noalloc(ctx, 0, 0, A, A, D)          # 48 * 2048 * 1024 bytes of slices > 64 MiB
    assert e.value.code == -1 and b"static device array" in H.lib().hsc_last_error()
    small = torch.zeros((1024, 640, 4), dtype=torch.float64, device=dev)
    Bm = torch.zeros((640, 1024, 4), dtype=torch.float64, device=dev)
    H.kern_zgemm_dd_noalloc(ctx, 0, 0, small, Bm, D)          # at the limit: accepted
    assert bool((D == 0).all())
