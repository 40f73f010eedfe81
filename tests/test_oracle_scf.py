"""Pins of the self-consistent NEGF-Poisson oracle (oracle/scf.py) against closed forms,
identities and brute-force stencil sums, none of which reuse the oracle's own arithmetic."""
import numpy as np
import pytest

import oracle
import synth

KW = dict(eta=1e-8, kT=0.025)


def _stencil_by_loops(u, grid, u_left, u_right):
    """sum over axes of (2 U_i - U_prev - U_next) with the ghost rules written out site by site"""
    nx, ny, nz = grid
    U = np.asarray(u).reshape(nz, ny, nx)
    out = np.zeros_like(U)
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                c = U[z, y, x]
                xm = U[z, y, x - 1] if x > 0 else u_left
                xp = U[z, y, x + 1] if x < nx - 1 else u_right
                ym = U[z, y - 1, x] if y > 0 else c
                yp = U[z, y + 1, x] if y < ny - 1 else c
                zm = U[z - 1, y, x] if z > 0 else c
                zp = U[z + 1, y, x] if z < nz - 1 else c
                out[z, y, x] = (2 * c - xm - xp) + (2 * c - ym - yp) + (2 * c - zm - zp)
    return out.reshape(-1)


def test_poisson_no_charge_is_the_linear_lead_to_lead_profile():
    grid = (7, 3, 4)
    u = oracle.scf.poisson_solve(grid, np.zeros(84), 0.3, -0.45)
    x = np.arange(84) % 7
    ref = 0.3 + (-0.45 - 0.3) * (x + 1) / 8.0
    assert np.abs(u - ref).max() < 1e-14


def test_poisson_separable_mode_closed_form():
    # sin along x (Dirichlet), cos of half-integer phase along y and z (Neumann): an eigenvector
    # of the stencil with eigenvalue sum over axes of 2 - 2 cos(theta)
    nx, ny, nz = 9, 5, 4
    kx, ky, kz = 3, 2, 1
    idx = np.arange(nx * ny * nz)
    x, y, z = idx % nx, (idx // nx) % ny, idx // (nx * ny)
    mode = (np.sin(np.pi * kx * (x + 1) / (nx + 1)) * np.cos(np.pi * ky * (y + 0.5) / ny) *
            np.cos(np.pi * kz * (z + 0.5) / nz))
    lam = (2 - 2 * np.cos(np.pi * kx / (nx + 1))) + (2 - 2 * np.cos(np.pi * ky / ny)) + (2 - 2 * np.cos(np.pi * kz / nz))
    u = oracle.scf.poisson_solve((nx, ny, nz), mode, 0.0, 0.0)
    assert np.abs(u - mode / lam).max() < 1e-13


@pytest.mark.parametrize("grid", [(3, 4, 2), (5, 1, 1), (1, 3, 3), (4, 4, 4)])
def test_poisson_residual_by_site_loops(grid):
    rng = np.random.default_rng(sum(grid))
    n = grid[0] * grid[1] * grid[2]
    rho = rng.normal(size=n)
    u = oracle.scf.poisson_solve(grid, rho, 0.7, -0.2)
    assert np.abs(_stencil_by_loops(u, grid, 0.7, -0.2) - rho).max() < 1e-12


def test_density_equilibrium_identity():
    # mu_L = mu_R: G^< = i f (A_L + A_R) and A_L + A_R = -2 Im G^r - A_eta, so the density from
    # G^< equals the f-weighted -Im G^r / pi less the eta broadening
    dev = synth.cuboid(5, 3, 2, onsite=np.random.default_rng(2).normal(0, 0.4, 30))
    E = np.linspace(-5.5, 5.5, 23)
    w = np.full(len(E), E[1] - E[0])
    out = oracle.dense.solve(dev, E, mu_L=0.2, mu_R=0.2, **KW)
    n_lesser = oracle.scf.density(w, out["gl"])
    f = oracle.negf.fermi(E, 0.2, KW["kT"])
    n_retarded = (w * f) @ (-2 * out["gr"].imag - out["a_eta"]) / (2 * np.pi)
    assert np.abs(n_lesser - n_retarded).max() < 1e-12 * np.abs(n_retarded).max()


def test_density_of_a_clean_chain_closed_form():
    # matched leads: every site of the chain sees the infinite chain, G_ii(z) = 1/sqrt(z^2 - 4 t^2)
    # (the root decaying for Im z > 0); the eta broadening inside the device is below 1e-6 here
    dev = synth.chain(6)
    E = np.linspace(-1.9, 1.9, 39)
    w = np.full(len(E), E[1] - E[0])
    out = oracle.dense.solve(dev, E, mu_L=0.0, mu_R=0.0, **KW)
    z = E + 1j * KW["eta"]
    g = 1 / np.sqrt(z * z - 4.0)
    g = np.where(g.imag > 0, -g, g)
    f = oracle.negf.fermi(E, 0.0, KW["kT"])
    ref = (w * f) @ (-g.imag / np.pi)
    n = oracle.scf.density(w, out["gl"])
    assert np.abs(n - ref).max() < 1e-6, (n, ref)


def test_potential_shift_moves_the_spectrum():
    # a uniform potential U0 shifts every level: G(E; U0) = G(E - U0; 0) when the leads move too;
    # with the leads fixed only the device moves, which a constant U on a single-site "device"
    # coupled to two leads shows in closed form: G = 1 / (z - U0 - 2 Sigma(z))
    dev = synth.chain(1)
    E = np.array([-1.3, 0.2, 0.9])
    out = oracle.dense.solve(dev, E, mu_L=0.0, mu_R=0.0, potential=np.array([0.37]), **KW)
    sig = oracle.negf.sigma_lead(E + 1j * KW["eta"], 0.0, -1.0, -1.0)
    ref = 1.0 / (E + 1j * KW["eta"] - 0.37 - 2 * sig)
    assert np.abs(out["gr"][:, 0] - ref).max() < 1e-14


def test_scf_without_coupling_is_the_laplace_profile():
    dev = synth.cuboid(4, 3, 2)
    E = np.linspace(-4, 4, 9)
    w = np.full(9, 1.0)
    r = oracle.scf.scf(dev, (4, 3, 2), E, w, 1e-8, 0.025, 0.1, -0.1, 0.2, -0.2, coupling=0.0, mixing=1.0,
                       iterations=2)
    x = np.arange(24) % 4
    assert np.abs(r["u"] - (0.2 - 0.4 * (x + 1) / 5)).max() < 1e-14
    assert r["residuals"][1] < 1e-14


def test_scf_fixed_point_and_screening_sign():
    dev = synth.cuboid(4, 3, 3, onsite=np.random.default_rng(5).normal(0, 0.2, 36))
    grid = (4, 3, 3)
    E = np.linspace(-6.0, 2.0, 33)
    w = np.full(33, E[1] - E[0])
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.05, mu_R=-0.05, u_left=0.0, u_right=0.0, coupling=0.2, mixing=0.6,
              iterations=60, tol=1e-12)
    r = oracle.scf.scf(dev, grid, E, w, **kw)
    assert r["residuals"][-1] < 1e-12 and len(r["residuals"]) < 60, r["residuals"]
    # the converged U solves Poisson with the density it produces (recomputed from scratch)
    dens = oracle.scf.density(w, oracle.dense.solve(dev, E, 1e-8, 0.05, 0.05, -0.05, potential=r["u"])["gl"])
    lhs = _stencil_by_loops(r["u"], grid, 0.0, 0.0)
    assert np.abs(lhs - 0.2 * dens).max() < 1e-9
    # electrons raise their own potential energy (repulsion): U > 0 inside, and a positive
    # background charge n0 lowers it
    assert r["u"].min() > 0
    r2 = oracle.scf.scf(dev, grid, E, w, n0=np.full(36, 0.05), **kw)
    assert (r2["u"] < r["u"]).all()


def test_anderson_without_history_is_linear_mixing():
    rng = np.random.default_rng(3)
    a = oracle.scf.Anderson(0, 0.4)
    x = rng.normal(size=7)
    for _ in range(4):
        gx = np.tanh(x) + 0.3
        nxt = a.step(x, gx)
        assert np.array_equal(nxt, x + 0.4 * (gx - x))
        x = nxt


def test_anderson_with_more_history_than_unknowns_restarts_linearly():
    # two unknowns and a history of four: the second difference already spans the space (the affine
    # map's fixed point is reached), and a third difference cannot be independent, so that step is
    # the linear one and the history restarts
    rng = np.random.default_rng(8)
    M = 0.5 * rng.normal(size=(2, 2))
    c = rng.normal(size=2)
    ref = np.linalg.solve(np.eye(2) - M, c)
    a = oracle.scf.Anderson(4, 0.5)
    x = np.array([0.3, -0.2])
    xs = [x]
    for _ in range(6):
        x = a.step(x, M @ x + c)
        xs.append(x)
    assert np.abs(xs[3] - ref).max() < 1e-12
    # the fourth step holds three differences of two unknowns: linear mixing, history cleared
    lin = xs[3] + 0.5 * (M @ xs[3] + c - xs[3])
    assert np.array_equal(xs[4], lin)
    assert np.abs(xs[-1] - ref).max() < 1e-12


def test_anderson_solves_an_affine_map_in_dimension_plus_one_steps():
    # for g(x) = M x + c Anderson mixing with enough history is GMRES on (I - M) x = c: it reaches the
    # fixed point (I - M)^-1 c after at most dim + 1 evaluations of g (here 6 unknowns)
    rng = np.random.default_rng(5)
    n = 6
    M = rng.normal(size=(n, n))
    M = 0.9 * M / np.abs(np.linalg.eigvals(M)).max()
    c = rng.normal(size=n)
    ref = np.linalg.solve(np.eye(n) - M, c)
    a = oracle.scf.Anderson(n, 1.0)
    x = np.zeros(n)
    for _ in range(n + 2):
        x = a.step(x, M @ x + c)
    assert np.abs(x - ref).max() < 1e-10 * np.abs(ref).max()
    # linear mixing needs far more steps for the same map
    y = np.zeros(n)
    lin = oracle.scf.Anderson(0, 1.0)
    for _ in range(n + 2):
        y = lin.step(y, M @ y + c)
    assert np.abs(y - ref).max() > 1e-3 * np.abs(ref).max()


def test_scf_with_anderson_mixing_reaches_the_same_fixed_point_sooner():
    dev = synth.cuboid(4, 3, 3, onsite=np.random.default_rng(5).normal(0, 0.2, 36))
    grid = (4, 3, 3)
    E = np.linspace(-6.0, 2.0, 33)
    w = np.full(33, E[1] - E[0])
    kw = dict(eta=1e-8, kT=0.05, mu_L=0.05, mu_R=-0.05, u_left=0.0, u_right=0.0, coupling=0.2, mixing=0.6,
              iterations=60, tol=1e-12)
    lin = oracle.scf.scf(dev, grid, E, w, **kw)
    acc = oracle.scf.scf(dev, grid, E, w, history=4, **kw)
    assert acc["residuals"][-1] < 1e-12 and len(acc["residuals"]) < len(lin["residuals"])
    assert np.abs(acc["u"] - lin["u"]).max() < 1e-11
