"""The closed-form eigenbases the device Poisson solve uploads (paper_1702_05167_amd/csrc/poisson_basis.h),
built with g++ for the host: Q is orthogonal and Q diag(lambda) Q^T is the 1D stencil 2 U_j - U_j-1 - U_j+1
with fixed outside values (Dirichlet, along x) or with the end point as its own outside neighbour (zero
normal derivative, along y and z), for sides from 1 to 64."""
import os
import shutil
import subprocess

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SIDES = (1, 2, 3, 7, 16, 32, 33, 64)


@pytest.fixture(scope="module")
def bases(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = tmp_path_factory.mktemp("pbasis") / "poisson_basis_driver"
    subprocess.run([gxx, "-std=c++17", "-O1", os.path.join(HERE, "native", "poisson_basis_driver.cpp"), "-o",
                    str(exe)], check=True, capture_output=True)
    cases = [(N, d) for N in SIDES for d in (1, 0)]
    out = subprocess.run([str(exe)], input="".join(f"{N} {d}\n" for N, d in cases), capture_output=True, text=True,
                         check=True).stdout.strip().splitlines()
    res = {}
    for (N, d), line in zip(cases, out):
        v = np.array([float(w) for w in line.split()])
        res[(N, d)] = (v[:N * N].reshape(N, N), v[N * N:])
    return res


def _stencil(N, dirichlet):
    T = 2.0 * np.eye(N) - np.eye(N, k=1) - np.eye(N, k=-1)
    if not dirichlet:
        T[0, 0] -= 1.0
        T[-1, -1] -= 1.0
    return T


@pytest.mark.parametrize("N", SIDES)
@pytest.mark.parametrize("dirichlet", [1, 0])
def test_basis_diagonalises_the_stencil(bases, N, dirichlet):
    Q, lam = bases[(N, dirichlet)]
    assert np.abs(Q.T @ Q - np.eye(N)).max() < 1e-13
    assert np.abs(Q @ np.diag(lam) @ Q.T - _stencil(N, dirichlet)).max() < 1e-13
    # the spectra: Dirichlet strictly positive, Neumann with the single zero mode (constant vector)
    if dirichlet:
        assert lam.min() > 0.0
    else:
        assert abs(lam[0]) < 1e-15 and (N == 1 or lam[1:].min() > 0.0)
        assert np.abs(Q[:, 0] - 1.0 / np.sqrt(N)).max() < 1e-15
