"""The two compute kernels in isolation: grouped complex GEMM and batched inverse.

Reference: plain PyTorch / NumPy CPU products and inverses in complex128.
"""
import numpy as np
import pytest
import torch

import paper_1702_05167_amd.hsc as H

pytestmark = pytest.mark.gpu


def _rand(rng, *shape):
    return rng.standard_normal(shape) + 1j * rng.standard_normal(shape)


def test_mfma_lane_layout(ctx):
    out = H.kern_mfma_probe(ctx).cpu().numpy().reshape(64, 4)
    A = np.zeros((16, 4))
    B = np.zeros((4, 16))
    for l in range(64):
        A[l % 16, l // 16] = 1.0 + l
        B[l // 16, l % 16] = 0.5 * ((l * 7) % 13) - 1.0
    D = A @ B
    exp = np.array([[D[l // 16 + 4 * r, l % 16] for r in range(4)] for l in range(64)])
    assert np.array_equal(out, exp)


OPS = [(a, b) for a in (0, 1, 2) for b in (0, 1, 2)]
SHAPES = [(1, 1, 1), (17, 33, 5), (64, 64, 16), (130, 70, 45), (65, 129, 1), (40, 50, 0), (200, 96, 300)]


def _op(x, o):
    return x if o == 0 else (x.T if o == 1 else x.conj().T)


@pytest.mark.parametrize("opA,opB", OPS)
@pytest.mark.parametrize("shape", SHAPES)
def test_zgemm_vs_cpu(ctx, opA, opB, shape):
    M, N, K = shape
    rng = np.random.default_rng(M * 1000 + N * 10 + K + 7 * opA + opB)
    a = _rand(rng, M, K) if opA == 0 else _rand(rng, K, M)
    b = _rand(rng, K, N) if opB == 0 else _rand(rng, N, K)
    c = _rand(rng, M, N)
    alpha = 0.75 - 1.25j
    dev = ctx.torch_device
    A, B, Cm = (torch.tensor(x, device=dev) for x in (a, b, c))
    for beta in (0, 1):
        D = H.kern_zgemm(ctx, opA, opB, alpha, A, B, beta=beta, C_=Cm if beta else None)
        ref = alpha * (_op(a, opA) @ _op(b, opB)) + (c if beta else 0)
        got = D.cpu().numpy()
        scale = max(1.0, np.abs(ref).max())
        assert np.abs(got - ref).max() <= 1e-13 * scale * max(1, K)


@pytest.mark.parametrize("tile", [1, 2, 3, 4, 5, 6, 7, 8])
@pytest.mark.parametrize("opA,opB", [(0, 0), (1, 0), (0, 2), (2, 1)])
@pytest.mark.parametrize("shape", [(1, 1, 1), (17, 33, 5), (130, 70, 45), (65, 129, 1), (200, 96, 300)])
def test_zgemm_tile_shapes(ctx, tile, opA, opB, shape):
    # tiles 1-3 sum k in the same order (steps of 4) as the default: equal bit for bit;
    # 4, 5, 7 use three real products per complex multiply-add, 6 and 7 the 4x4x4 MFMA
    M, N, K = shape
    rng = np.random.default_rng(M * 7 + N * 3 + K + tile)
    a = _rand(rng, M, K) if opA == 0 else _rand(rng, K, M)
    b = _rand(rng, K, N) if opB == 0 else _rand(rng, N, K)
    c = _rand(rng, M, N)
    dev = ctx.torch_device
    A, B, Cm = (torch.tensor(x, device=dev) for x in (a, b, c))
    D0 = H.kern_zgemm(ctx, opA, opB, 0.5 + 2j, A, B, beta=1, C_=Cm, tile=0)
    D1 = H.kern_zgemm(ctx, opA, opB, 0.5 + 2j, A, B, beta=1, C_=Cm, tile=tile)
    ref = (0.5 + 2j) * (_op(a, opA) @ _op(b, opB)) + c
    tol = (1e-13 if tile in (1, 2, 3, 6, 8) else 3e-13) * max(1.0, np.abs(ref).max()) * max(1, K)
    assert np.abs(D1.cpu().numpy() - ref).max() <= tol
    if tile in (1, 2, 3, 8):
        assert torch.equal(D0, D1)


def test_zgemm_inplace_leading_dims(ctx):
    rng = np.random.default_rng(3)
    big = _rand(rng, 150, 160)
    dev = ctx.torch_device
    T = torch.tensor(big, device=dev)
    A = T[10:80, 5:25]          # 70 x 20, ld 160
    B = T[100:120, 30:121]      # 20 x 91
    D = T[0:70, 60:151]         # in place on a sub-block
    ref = big.copy()
    ref[0:70, 60:151] = big[10:80, 5:25] @ big[100:120, 30:121] + big[0:70, 60:151]
    H.kern_zgemm(ctx, 0, 0, 1.0, A, B, beta=1, C_=D, D=D)
    assert np.abs(T.cpu().numpy() - ref).max() < 1e-12


@pytest.mark.parametrize("sizes", [[1, 2, 5], [31, 64, 100], [300, 513], [1024]])
def test_zinv_batched_vs_cpu(ctx, sizes):
    rng = np.random.default_rng(sum(sizes))
    dev = ctx.torch_device
    host = [_rand(rng, n, n) + 2.0 * np.eye(n) for n in sizes]
    mats = [torch.tensor(h, device=dev) for h in host]
    inv, st = H.kern_zinv_batched(ctx, mats)
    assert st.cpu().numpy().tolist() == [0] * len(sizes)
    for h, g in zip(host, inv):
        ref = np.linalg.inv(h)
        err = np.abs(g.cpu().numpy() - ref).max() / np.abs(ref).max()
        assert err < 1e-11 * np.linalg.cond(h)


def test_zinv_needs_pivoting(ctx):
    # zero leading diagonal: only row interchanges make Gauss-Jordan work
    n = 48
    rng = np.random.default_rng(11)
    h = _rand(rng, n, n)
    h[np.arange(n), np.arange(n)] = 0.0
    inv, st = H.kern_zinv_batched(ctx, [torch.tensor(h, device=ctx.torch_device)])
    assert int(st[0]) == 0
    ref = np.linalg.inv(h)
    assert np.abs(inv[0].cpu().numpy() - ref).max() / np.abs(ref).max() < 1e-10


def test_zinv_singular_reports_status(ctx):
    h = np.zeros((4, 4), complex)
    inv, st = H.kern_zinv_batched(ctx, [torch.tensor(h, device=ctx.torch_device)])
    assert int(st[0]) == H.HscError(-3, "").code
    assert np.isfinite(inv[0].cpu().numpy()).all()


# ---- the double-double block product (precision >= 1) against exact rational arithmetic ----

def _dd_rand(rng, rows, cols):
    """(rows, cols, 4) double-double values: hi ~ N(0, 1), lo a random fraction of half an ulp of hi"""
    hi = rng.standard_normal((rows, cols, 2))
    lo = (rng.random((rows, cols, 2)) - 0.5) * np.spacing(np.abs(hi))
    out = np.empty((rows, cols, 4))
    out[..., 0], out[..., 1], out[..., 2], out[..., 3] = hi[..., 0], lo[..., 0], hi[..., 1], lo[..., 1]
    return out


def _dd_exact(x):
    """(re, im) as exact rationals of one double-double element"""
    from fractions import Fraction as F
    return F(float(x[0])) + F(float(x[1])), F(float(x[2])) + F(float(x[3]))


@pytest.mark.parametrize("config", [0, 1, 2])
@pytest.mark.parametrize("opA,opB,negate,beta", [(0, 0, 0, 0), (1, 0, 1, 1), (0, 1, 0, 1)])
def test_zgemm_dd_against_exact_arithmetic(ctx, config, opA, opB, negate, beta):
    # ragged sizes spanning several tiles of every configuration; error measured against the exact
    # (rational) value, relative to sum_k |a_ik| |b_kj| + |c_ij|: double-double gives ~1e-31 there,
    # complex128 arithmetic (or error-free transformations broken by contraction) ~1e-16
    rng = np.random.default_rng(10 * config + 3 * opA + opB)
    M, N, K = 70, 37, 45
    A = _dd_rand(rng, *((M, K) if opA == 0 else (K, M)))
    B = _dd_rand(rng, *((K, N) if opB == 0 else (N, K)))
    Cm = _dd_rand(rng, M, N)
    dev = ctx.torch_device
    D = H.kern_zgemm_dd(ctx, opA, opB, torch.tensor(A, device=dev), torch.tensor(B, device=dev), negate=negate,
                        beta=beta, C_=torch.tensor(Cm, device=dev) if beta else None, config=config).cpu().numpy()
    # the stored pairs are normalised: |lo| <= ulp(hi) / 2
    assert (np.abs(D[..., 1]) <= 0.5 * np.spacing(np.abs(D[..., 0]))).all()
    assert (np.abs(D[..., 3]) <= 0.5 * np.spacing(np.abs(D[..., 2]))).all()
    # exact values at the tile corners and at 60 random entries
    pairs = {(i, j) for i in (0, 31, 32, 63, 64, M - 1) for j in (0, 31, 32, N - 1)}
    pairs |= {(int(i), int(j)) for i, j in zip(rng.integers(0, M, 60), rng.integers(0, N, 60))}
    worst = 0.0
    for i, j in sorted(pairs):
        re = im = 0
        scale = 0.0
        for k in range(K):
            ar, ai = _dd_exact(A[i, k] if opA == 0 else A[k, i])
            br, bi = _dd_exact(B[k, j] if opB == 0 else B[j, k])
            re += ar * br - ai * bi
            im += ar * bi + ai * br
            scale += abs(complex(float(ar), float(ai))) * abs(complex(float(br), float(bi)))
        if negate:
            re, im = -re, -im
        if beta:
            cr, ci = _dd_exact(Cm[i, j])
            re, im = re + cr, im + ci
            scale += abs(complex(float(cr), float(ci)))
        got = _dd_exact(D[i, j])
        err = max(abs(float(got[0] - re)), abs(float(got[1] - im))) / scale
        worst = max(worst, err)
    print("dd GEMM worst relative error", worst)
    assert worst < 1e-29


@pytest.mark.parametrize("matrix_cores", [0, 1])
def test_zinv_dd_nearly_singular_block(ctx, matrix_cores):
    # a complex-symmetric block like the fold's pivot blocks out of the lead band: real symmetric with one
    # eigenvalue at 1e-10 plus i 1e-12 (condition ~3e10).  The double-double Gauss-Jordan inverse must
    # satisfy A Y = I to ~kappa 1e-31 in exact arithmetic; the complex128 one only to ~kappa 1e-16
    from fractions import Fraction as F
    rng = np.random.default_rng(5)
    n = 24
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([[1e-10], rng.uniform(1.0, 3.0, n - 1) * rng.choice([-1.0, 1.0], n - 1)])
    R = (Q * lam) @ Q.T
    R = 0.5 * (R + R.T)
    A = R + 1j * 1e-12 * np.eye(n)
    Xd = np.zeros((n, n, 4))
    Xd[..., 0], Xd[..., 2] = A.real, A.imag
    Y, st = H.kern_zinv_dd(ctx, torch.tensor(Xd, device=ctx.torch_device), matrix_cores=matrix_cores)
    Y = Y.cpu().numpy()
    assert int(st.cpu()[0]) == 0
    Ax = [[(F(float(A[i, j].real)), F(float(A[i, j].imag))) for j in range(n)] for i in range(n)]
    Yx = [[(F(float(Y[i, j, 0])) + F(float(Y[i, j, 1])), F(float(Y[i, j, 2])) + F(float(Y[i, j, 3])))
           for j in range(n)] for i in range(n)]
    ynorm = max(abs(complex(float(a), float(b))) for row in Yx for a, b in row)
    worst = 0.0
    for i in range(n):
        for j in range(n):
            re = im = F(0)
            for k in range(n):
                ar, ai = Ax[i][k]
                yr, yi = Yx[k][j]
                re += ar * yr - ai * yi
                im += ar * yi + ai * yr
            if i == j:
                re -= 1
            worst = max(worst, abs(float(re)), abs(float(im)))
    Y64, _ = H.kern_zinv_batched(ctx, [torch.tensor(A, device=ctx.torch_device)])
    r64 = np.abs(A @ Y64[0].cpu().numpy() - np.eye(n)).max()
    print("residual max |A Y - I|: double-double", worst, "complex128", r64, "max |Y|", ynorm)
    assert ynorm > 1e9                       # the block is as nearly singular as intended
    assert worst < 1e-18 and worst < r64 * 1e-8
